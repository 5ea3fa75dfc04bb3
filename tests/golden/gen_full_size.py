"""Write full-size expected values computed by the CPU oracle only.

Usage: python tests/golden/gen_full_size.py [name ...]
Each entry records the workload recipe, the oracle's f and norm, and the
wall time it took.  Inputs come from workloads/ (seeded); values from oracle/.

The *_amplitudes entries go to full_size_amplitudes.json: psi_p of the
oracle at AMP_SAMPLES seeded indices plus a few structured ones (see
sample_indices), as (index, re, im).
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import (CONFIG_SEEDS, qaoa_maxcut_workload, qwoa_constrained_workload,  # noqa: E402
                       qwoa_portfolio_workload)

OUT = os.path.join(HERE, "full_size_values.json")
OUT_AMP = os.path.join(HERE, "full_size_amplitudes.json")
AMP_SAMPLES = 4096
AMP_SEED = 2028


def sample_indices(N: int) -> np.ndarray:
    """AMP_SAMPLES distinct indices drawn by default_rng(AMP_SEED), plus 0, 1,
    the top index, the middle and every single-bit index (sorted, unique)."""
    rng = np.random.default_rng(AMP_SEED)
    idx = set(int(i) for i in rng.choice(N, AMP_SAMPLES, replace=False))
    idx |= {0, 1, N - 1, N // 2}
    idx |= {1 << b for b in range(N.bit_length() - 1)}
    return np.array(sorted(idx), dtype=np.int64)


def _amp_entry(recipe, psi, f, nrm, secs):
    idx = sample_indices(len(psi))
    v = psi[idx]
    return {"recipe": recipe, "f": f, "norm": nrm, "oracle_seconds": secs,
            "oracle_threads": oracle.get_threads(),
            "index_rule": f"sample_indices(N): default_rng({AMP_SEED}).choice(N, {AMP_SAMPLES}, replace=False) "
                          "| {0, 1, N-1, N//2, 2^b}",
            "index": [int(i) for i in idx], "re": [float(x) for x in v.real], "im": [float(x) for x in v.imag]}


def qaoa_n28_amplitudes():
    wl = qaoa_maxcut_workload(28, 8, graph="regular3", weighted=True, seed=CONFIG_SEEDS["qaoa_n28"])
    t0 = time.time()
    psi, f, nrm = oracle.evolve("x", wl.q, wl.gammas, wl.ts)
    return _amp_entry("qaoa_maxcut_workload(28, 8, graph='regular3', weighted=True, seed=102); psi_p",
                      psi, f, nrm, time.time() - t0)


def qwoa_n26_amplitudes():
    wl = qwoa_portfolio_workload(26, 6, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="ring")
    lam = oracle.ring_lambda(wl.N)
    t0 = time.time()
    psi, f, nrm = oracle.evolve("circulant", wl.q, wl.gammas, wl.ts, lam)
    return _amp_entry("qwoa_portfolio_workload(26, 6, seed=103, lambda_kind='ring'); psi_p",
                      psi, f, nrm, time.time() - t0)


def qaoa_n28():
    wl = qaoa_maxcut_workload(28, 8, graph="regular3", weighted=True, seed=CONFIG_SEEDS["qaoa_n28"])
    t0 = time.time()
    _, f, nrm = oracle.evolve("x", wl.q, wl.gammas, wl.ts)
    return {"recipe": "qaoa_maxcut_workload(28, 8, graph='regular3', weighted=True, seed=102)",
            "f": f, "norm": nrm, "oracle_seconds": time.time() - t0}


def qwoa_n26():
    wl = qwoa_portfolio_workload(26, 6, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="ring")
    lam = oracle.ring_lambda(wl.N)
    t0 = time.time()
    _, f, nrm = oracle.evolve("circulant", wl.q, wl.gammas, wl.ts, lam)
    return {"recipe": "qwoa_portfolio_workload(26, 6, seed=103, lambda_kind='ring')",
            "f": f, "norm": nrm, "oracle_seconds": time.time() - t0}


def qwoa_n26_complete():
    # the complete graph's mixer from its definition (closed form): the
    # transform route would round t (N - 1) for the eigenvalue N - 1
    wl = qwoa_portfolio_workload(26, 6, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="complete")
    t0 = time.time()
    _, f, nrm = oracle.evolve("complete", wl.q, wl.gammas, wl.ts)
    secs = time.time() - t0
    # the same spectrum through the transform route (eigenvalue array)
    _, f_tr, _ = oracle.evolve("circulant", wl.q, wl.gammas, wl.ts, oracle.complete_lambda(wl.N))
    return {"recipe": "qwoa_portfolio_workload(26, 6, seed=103, lambda_kind='complete')",
            "f": f, "norm": nrm, "oracle_seconds": secs, "f_transform": f_tr}


def qwoa_n26_complete_grad():
    wl = qwoa_portfolio_workload(26, 6, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="complete")
    t0 = time.time()
    f, dg, dt = oracle.grad("complete", wl.q, wl.gammas, wl.ts)
    return {"recipe": "qwoa_portfolio_workload(26, 6, seed=103, lambda_kind='complete'); oracle.grad",
            "f": f, "dgammas": list(map(float, dg)), "dts": list(map(float, dt)),
            "oracle_seconds": time.time() - t0}


def qwoa_m26_k13_ring():
    # N = C(26, 13) = 10,400,600 = 2^3 5^2 7 17 19 23: the oracle's chirp-z route
    wl = qwoa_constrained_workload(26, 13, 6, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="ring")
    t0 = time.time()
    psi, f, nrm = oracle.evolve("circulant", wl.q, wl.gammas, wl.ts, oracle.ring_lambda(wl.N))
    return _amp_entry("qwoa_constrained_workload(26, 13, 6, seed=103, lambda_kind='ring'); psi_p",
                      psi, f, nrm, time.time() - t0)


# A smooth N = 2^3 3^5 5^3 7^2 = 11,907,000 with seeded qualities and angles
SMOOTH_N = 2 ** 3 * 3 ** 5 * 5 ** 3 * 7 ** 2
SMOOTH_SEED = 2029


def smooth_inputs(p: int):
    rng = np.random.default_rng(SMOOTH_SEED)
    q = rng.uniform(-1.0, 3.0, SMOOTH_N)
    return q, rng.uniform(0, np.pi, p), rng.uniform(0, np.pi, p)


def smooth_ring_grad():
    q, g, t = smooth_inputs(2)
    t0 = time.time()
    f, dg, dt = oracle.grad("circulant", q, g, t, oracle.ring_lambda(SMOOTH_N))
    return {"recipe": f"N = {SMOOTH_N}; default_rng({SMOOTH_SEED}): q ~ U(-1, 3) over N, then gammas, ts "
                      "~ U(0, pi), p = 2; ring; oracle.grad",
            "f": f, "dgammas": list(map(float, dg)), "dts": list(map(float, dt)),
            "oracle_seconds": time.time() - t0}


GENERATORS = {"qaoa_n28_p8": qaoa_n28, "qwoa_n26_p6": qwoa_n26, "qwoa_n26_p6_complete": qwoa_n26_complete,
              "qwoa_n26_p6_complete_grad": qwoa_n26_complete_grad,
              "qaoa_n28_p8_amplitudes": qaoa_n28_amplitudes, "qwoa_n26_p6_amplitudes": qwoa_n26_amplitudes,
              "qwoa_m26_k13_p6_ring_amplitudes": qwoa_m26_k13_ring, "smooth_11907000_p2_ring_grad": smooth_ring_grad}


def main(names):
    for name in names or GENERATORS:
        out = OUT_AMP if name.endswith("_amplitudes") else OUT
        data = {}
        if os.path.exists(out):
            with open(out) as fh:
                data = json.load(fh)
        print(f"computing {name} ...", flush=True)
        data[name] = GENERATORS[name]()
        print(name, {k: v for k, v in data[name].items() if k not in ("index", "re", "im")}, flush=True)
        with open(out, "w") as fh:
            json.dump(data, fh, indent=None if out == OUT_AMP else 1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
