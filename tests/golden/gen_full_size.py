"""Write full-size expected values computed by the CPU oracle only.

Usage: python tests/golden/gen_full_size.py [name ...]
Each entry records the workload recipe, the oracle's f and norm, and the
wall time it took.  Inputs come from workloads/ (seeded); values from oracle/.
"""

from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import CONFIG_SEEDS, qaoa_maxcut_workload, qwoa_portfolio_workload  # noqa: E402

OUT = os.path.join(HERE, "full_size_values.json")


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


GENERATORS = {"qaoa_n28_p8": qaoa_n28, "qwoa_n26_p6": qwoa_n26, "qwoa_n26_p6_complete": qwoa_n26_complete,
              "qwoa_n26_p6_complete_grad": qwoa_n26_complete_grad}


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    for name in names or GENERATORS:
        print(f"computing {name} ...", flush=True)
        data[name] = GENERATORS[name]()
        print(name, data[name], flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
