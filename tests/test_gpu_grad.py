"""GPU parity: adjoint gradient (qva_grad) vs the CPU oracle.

Bar: ||g - g_ref||_inf / ||g_ref||_inf <= 1e-10 against the oracle's adjoint
gradient (itself pinned to a brute-force product-rule gradient and to central
differences on the CPU), f to 1e-12 relative.  Full-size pins at n = 30: the
p = 1 ring closed form and the ring light cone (f/n and g/n do not depend on
n once n >= 2p + 2).
"""

import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from gpu_util import to_dev  # noqa: E402
from workloads import (CONFIG_SEEDS, maxcut_qualities, qaoa_maxcut_workload,  # noqa: E402
                       random_symmetric_lambda, ring_cut_qualities_device, ring_edges)

pytestmark = pytest.mark.gpu
qva = pytest.importorskip("paper_2110_03963_amd")

G_TOL = 1e-10
F_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qva.load_library()


def _gerr(dg, dt, rg, rt):
    g = np.concatenate([dg, dt])
    r = np.concatenate([rg, rt])
    return float(np.max(np.abs(g - r)) / max(np.max(np.abs(r)), 1e-300))


def _check(mixer, q, g, t, lam=None, kind="array"):
    if mixer == "x":
        prob = qva.Problem(to_dev(q), "x")
    else:
        prob = qva.Problem(to_dev(q), "circulant", to_dev(lam) if kind == "array" else None, kind)
        lam = oracle.lambda_for(kind, len(q), lam)
    f, dg, dt = qva.grad(prob, g, t)
    if mixer == "circulant" and kind == "complete":  # the oracle's closed form
        f_ref, rg, rt = oracle.grad("complete", q, g, t)
    else:
        f_ref, rg, rt = oracle.grad(mixer, q, g, t, lam)
    assert abs(f.item() - f_ref) <= F_TOL * max(abs(f_ref), np.mean(np.abs(q)))
    err = _gerr(dg.cpu().numpy(), dt.cpu().numpy(), rg, rt)
    assert err < G_TOL, err
    return f.item(), dg.cpu().numpy(), dt.cpu().numpy()


@pytest.mark.parametrize("n,p", [(1, 1), (3, 2), (8, 4), (12, 3), (13, 1), (13, 3), (14, 2),
                                 (17, 3), (20, 2), (21, 4), (22, 2), (23, 3)])
def test_grad_x(n, p):
    rng = np.random.default_rng(31 * n + p)
    q = rng.uniform(0, 5, 1 << n)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    _check("x", q, g, t)


@pytest.mark.parametrize("n,p", [(2, 2), (6, 3), (12, 2), (13, 2), (15, 3), (21, 2), (22, 2)])
@pytest.mark.parametrize("kind", ["ring", "complete", "array"])
def test_grad_circulant(n, p, kind):
    rng = np.random.default_rng(17 * n + p + len(kind))
    N = 1 << n
    q = rng.uniform(-2, 3, N)
    lam = random_symmetric_lambda(N, rng) if kind == "array" else None
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    _check("circulant", q, g, t, lam, kind)


@pytest.mark.parametrize("n,p", [(13, 1), (16, 3), (20, 4)])
def test_grad_complete_closed_form(n, p):
    """Complete graph, n > 12: the closed-form adjoint passes against the
    oracle's closed-form adjoint (f to 1e-12, gradient to 1e-10); at n = 20
    the transform route would already be off by ~1e-10 (eigenvalue N - 1)."""
    rng = np.random.default_rng(5 * n + p)
    N = 1 << n
    q = rng.uniform(-1, 3, N)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    f, dg, dt = _check("circulant", q, g, t, None, "complete")
    # repeatable bit for bit
    prob = qva.Problem(to_dev(q), "circulant", None, "complete")
    f2, dg2, dt2 = qva.grad(prob, g, t)
    assert f2.item() == f and np.array_equal(dg2.cpu().numpy(), dg) and np.array_equal(dt2.cpu().numpy(), dt)


@pytest.mark.parametrize("N,p", [(7, 2), (5000, 3), (200003, 4), (1000003, 2)])
def test_grad_complete_any_n(N, p):
    """Closed-form adjoint on N solutions, N not a power of two, against the
    oracle's closed-form adjoint."""
    rng = np.random.default_rng(N + p)
    q = rng.uniform(-1, 3, N)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    prob = qva.Problem(to_dev(q), "circulant", None, "complete")
    f, dg, dt = qva.grad(prob, g, t)
    f_ref, rg, rt = oracle.grad("complete", q, g, t)
    assert abs(f.item() - f_ref) <= F_TOL * max(abs(f_ref), np.mean(np.abs(q)))
    assert _gerr(dg.cpu().numpy(), dt.cpu().numpy(), rg, rt) < G_TOL


@pytest.mark.parametrize("N,p,kind", [(1000, 2, "ring"), (4097, 3, "array"), (100003, 2, "ring"),
                                      (100003, 1, "array"), (3000017, 2, "ring")])
def test_grad_bluestein_any_n(N, p, kind):
    """Adjoint through Bluestein's transform (ring or eigenvalue array over N
    solutions, N not a power of two) against the oracle's adjoint, which is
    pinned to the brute-force product rule and central differences."""
    rng = np.random.default_rng(N + 7 * p)
    q = rng.uniform(-1, 3, N)
    lam = rng.uniform(-2, 2, N) if kind == "array" else None
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    print(f"bluestein grad N={N} p={p} {kind}", flush=True)
    _check("circulant", q, g, t, lam, kind)
    prob = qva.Problem(to_dev(q), "circulant", to_dev(lam) if kind == "array" else None, kind)
    fe, _, _ = qva.evolve(prob, g, t, store=False)
    fg, _, _ = qva.grad(prob, g, t)
    assert abs(fe.item() - fg.item()) <= 1e-13 * np.mean(np.abs(q))


def test_grad_n12_regular3_p12():
    """The adjoint-gradient workload's oracle-parity size: weighted 3-regular
    MaxCut, n = 12, p = 12 (24 parameters)."""
    wl = qaoa_maxcut_workload(12, 12, graph="regular3", weighted=True, seed=CONFIG_SEEDS["grad_n30"])
    f, dg, dt = _check("x", wl.q, wl.gammas, wl.ts)
    bg, bt = oracle.grad_bruteforce("x", wl.q, wl.gammas, wl.ts)
    assert _gerr(dg, dt, bg, bt) < G_TOL


def test_grad_matches_bruteforce_tiled():
    """n = 14 (tile passes), compared with the oracle's product-rule gradient."""
    rng = np.random.default_rng(2)
    q = rng.uniform(0, 3, 1 << 14)
    g = rng.uniform(0, math.pi, 3)
    t = rng.uniform(0, math.pi, 3)
    _, dg, dt = _check("x", q, g, t)
    bg, bt = oracle.grad_bruteforce("x", q, g, t)
    assert _gerr(dg, dt, bg, bt) < G_TOL


def _central_differences(prob, g, t, h=1e-5):
    """Central differences of the GPU forward, with the step actually taken,
    (x + h) - (x - h), as the denominator."""
    p = len(g)
    fd = []
    for which in (0, 1):
        for k in range(p):
            gp, gm, tp, tm = g.copy(), g.copy(), t.copy(), t.copy()
            if which == 0:
                gp[k] += h
                gm[k] -= h
                step = gp[k] - gm[k]
            else:
                tp[k] += h
                tm[k] -= h
                step = tp[k] - tm[k]
            fp = qva.evolve(prob, gp, tp, store=False)[0].item()
            fm = qva.evolve(prob, gm, tm, store=False)[0].item()
            fd.append((fp - fm) / step)
    return np.array(fd)


def test_c4_weighted_n30_p12_adjoint_vs_central_differences():
    """The adjoint workload at full size: weighted random 3-regular MaxCut,
    n = 30, p = 12 (24 parameters).  The adjoint gradient against central
    differences of the GPU forward with h = 1e-5:
    max |g_adj - g_fd| <= 1e-8 max |g_adj|."""
    from workloads import maxcut_qualities_device

    n, p = 30, 12
    print("adjoint n=30 p=12 vs central differences", flush=True)
    wl = qaoa_maxcut_workload(n, p, graph="regular3", weighted=True, seed=CONFIG_SEEDS["grad_n30"],
                              build_q=False)
    prob = qva.Problem(maxcut_qualities_device(n, wl.edges, wl.weights, "cuda"), "x")
    g = np.asarray(wl.gammas, np.float64)
    t = np.asarray(wl.ts, np.float64)
    f, dg, dt = qva.grad(prob, g, t)
    ad = np.concatenate([dg.cpu().numpy(), dt.cpu().numpy()])
    torch.cuda.empty_cache()  # the forward needs one state, not two
    fd = _central_differences(prob, g, t)
    rel = float(np.max(np.abs(ad - fd)) / np.max(np.abs(ad)))
    print(f"  max |g_adj - g_fd| / max |g_adj| = {rel:.3e}", flush=True)
    assert rel <= 1e-8, rel
    f_ev = qva.evolve(prob, g, t, store=False)[0].item()
    assert abs(f.item() - f_ev) <= 1e-13 * abs(f_ev)
    del prob
    torch.cuda.empty_cache()


def test_grad_vs_central_differences_gpu():
    """Central differences of the GPU forward (h = 1e-5) agree to 1e-8."""
    rng = np.random.default_rng(4)
    n, p = 16, 3
    q = rng.uniform(0, 3, 1 << n)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    prob = qva.Problem(to_dev(q), "x")
    _, dg, dt = qva.grad(prob, g, t)
    fd = _central_differences(prob, g, t)
    ad = np.concatenate([dg.cpu().numpy(), dt.cpu().numpy()])
    assert np.max(np.abs(ad - fd)) <= 1e-8 * np.max(np.abs(ad))


def test_grad_f_equals_evolve_f():
    rng = np.random.default_rng(6)
    n = 20
    q = rng.uniform(0, 3, 1 << n)
    prob = qva.Problem(to_dev(q), "x")
    g, t = [0.3, 1.7, 0.9], [2.2, 0.4, 1.1]
    f1 = qva.grad(prob, g, t)[0].item()
    f2 = qva.evolve(prob, g, t, store=False)[0].item()
    assert abs(f1 - f2) < 1e-13 * abs(f2)


def test_grad_depth_zero():
    rng = np.random.default_rng(8)
    q = rng.uniform(0, 3, 1 << 15)
    prob = qva.Problem(to_dev(q), "x")
    f, dg, dt = qva.grad(prob, [], [])
    assert dg.numel() == 0 and dt.numel() == 0
    assert abs(f.item() - q.mean()) < 1e-13 * q.mean()


def test_ring_p1_closed_form_full_size():
    """n = 30 (16 GiB per vector), unweighted ring, p = 1:
    df/dgamma = (n/2) sin 4t cos 2gamma, df/dt = n cos 4t sin 2gamma."""
    n = 30
    prob = qva.Problem(ring_cut_qualities_device(n, "cuda"), "x")
    gam, tt = 0.43, 1.21
    f, dg, dt = qva.grad(prob, [gam], [tt])
    assert abs(f.item() - n * (0.5 + 0.25 * math.sin(4 * tt) * math.sin(2 * gam))) < 1e-12 * n
    assert abs(dg.item() - n / 2 * math.sin(4 * tt) * math.cos(2 * gam)) < 1e-10 * n
    assert abs(dt.item() - n * math.cos(4 * tt) * math.sin(2 * gam)) < 1e-10 * n


@pytest.mark.parametrize("n", [29, 30, 31])
def test_ring_light_cone_gradient_full_size(n):
    """Unweighted ring, p = 3: f/n and grad/n equal the oracle's at n = 8.
    n = 29 has one 3-column and one 4-column strided group, n = 30 two
    3-column groups (rotation of element bit 3 across lanes), n = 31 three
    strided groups."""
    p = 3
    rng = np.random.default_rng(12)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    ns = 2 * p + 2
    f_s, g_s, t_s = oracle.grad("x", oracle.maxcut_quality_loop(ns, ring_edges(ns)), g, t)
    print(f"ring light cone gradient n={n}", flush=True)
    prob = qva.Problem(ring_cut_qualities_device(n, "cuda"), "x")
    f, dg, dt = qva.grad(prob, g, t)
    assert abs(f.item() / n - f_s / ns) < 1e-12 * abs(f_s / ns)
    err = _gerr(dg.cpu().numpy() / n, dt.cpu().numpy() / n, g_s / ns, t_s / ns)
    assert err < G_TOL
    del prob
    torch.cuda.empty_cache()


def test_ring_light_cone_gradient_max_size():
    """n = 32, the largest register whose two gradient vectors fit (2 x 64 GiB
    plus 32 GiB of q), unweighted ring, p = 2: f/n and grad/n equal the
    oracle's at n = 6."""
    p = 2
    rng = np.random.default_rng(32)
    g = rng.uniform(0, math.pi, p)
    t = rng.uniform(0, math.pi, p)
    ns = 2 * p + 2
    f_s, g_s, t_s = oracle.grad("x", oracle.maxcut_quality_loop(ns, ring_edges(ns)), g, t)
    n = 32
    print("max size gradient n=32", flush=True)
    prob = qva.Problem(ring_cut_qualities_device(n, "cuda"), "x")
    f, dg, dt = qva.grad(prob, g, t)
    assert abs(f.item() / n - f_s / ns) < 1e-12 * abs(f_s / ns)
    err = _gerr(dg.cpu().numpy() / n, dt.cpu().numpy() / n, g_s / ns, t_s / ns)
    assert err < G_TOL
    del prob
    torch.cuda.empty_cache()


def test_autograd_function():
    rng = np.random.default_rng(10)
    n, p = 14, 2
    q = rng.uniform(0, 3, 1 << n)
    prob = qva.Problem(to_dev(q), "x")
    g = torch.tensor(rng.uniform(0, 3, p), dtype=torch.float64, device="cuda", requires_grad=True)
    t = torch.tensor(rng.uniform(0, 3, p), dtype=torch.float64, device="cuda", requires_grad=True)
    f = qva.expectation_value(prob, g, t)
    (3.0 * f).backward()
    f_ref, rg, rt = oracle.grad("x", q, g.detach().cpu().numpy(), t.detach().cpu().numpy())
    assert abs(f.item() - f_ref) < 1e-12 * f_ref
    assert _gerr(g.grad.cpu().numpy(), t.grad.cpu().numpy(), 3 * rg, 3 * rt) < G_TOL
