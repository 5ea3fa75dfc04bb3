"""The oracle's results do not depend on its thread count.

OpenMP splits only loops whose iterations write their own elements; every
sum stays a single-threaded pairwise sum.  So states, f and gradients must be
bit-identical at 1 thread and at several, for every mixer and both the
forward evolution and the adjoint.
"""

import math

import numpy as np
import pytest

import oracle


def _run_both(fn):
    before = oracle.get_threads()
    try:
        oracle.set_threads(1)
        a = fn()
        oracle.set_threads(4)
        b = fn()
    finally:
        oracle.set_threads(before)
    return a, b


def _same(a, b):
    for x, y in zip(a, b):
        x = np.atleast_1d(np.asarray(x))
        y = np.atleast_1d(np.asarray(y))
        assert x.shape == y.shape
        assert x.tobytes() == y.tobytes()


@pytest.fixture(scope="module")
def setup():
    rng = np.random.default_rng(11)
    return rng


@pytest.mark.parametrize("mixer,N", [("x", 1 << 14), ("circulant", 1 << 13), ("circulant", 5003),
                                     ("complete", 6000)])
def test_evolve_and_grad_thread_independent(setup, mixer, N):
    rng = setup
    q = rng.uniform(-1, 3, N)
    g = rng.uniform(0, math.pi, 3)
    t = rng.uniform(0, math.pi, 3)
    lam = oracle.ring_lambda(N) if mixer == "circulant" else None
    _same(*_run_both(lambda: oracle.evolve(mixer, q, g, t, lam)))
    _same(*_run_both(lambda: oracle.grad(mixer, q, g, t, lam)))


def test_terms_and_xy_thread_independent(setup):
    rng = setup
    n = 12
    q = rng.uniform(0, 3, 1 << n)
    support = [3, 5, 0x81, 0x700]
    coef = rng.uniform(-1, 1, 4)
    g = rng.uniform(0, 1, (2, 4))
    t = rng.uniform(0, 1, 2)
    _same(*_run_both(lambda: oracle.grad_terms(q, support, coef, g, t)))
    pairs = oracle.parity_ring_pairs(list(range(n)))
    psi0 = np.zeros(1 << n, np.complex128)
    psi0[0b000000111111] = 1.0
    _same(*_run_both(lambda: oracle.grad_xy(q, psi0, pairs, g[:, 0], t)))


def test_fft_thread_independent(setup):
    x = setup.standard_normal(1 << 15) + 1j * setup.standard_normal(1 << 15)
    _same(*_run_both(lambda: (oracle.fft(x, -1), oracle.bluestein(x[:7001], +1))))
