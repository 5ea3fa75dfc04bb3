"""Seeded synthetic inputs for the QVA state-evolution path.

This package builds problem *inputs* only: graphs, edge weights, the quality
vector q of a combinatorial problem, circulant eigenvalue vectors and the
variational parameters (gamma, t).  It contains none of the evolution's
arithmetic (no phase, mixer, Fourier transform or expectation), so both the
CPU oracle and the GPU path can consume exactly the same bytes.

Conventions (paper, Sec. 2.2 and 5.1):
  * basis index j of an n-qubit register, bit i of j is the value of qubit i
    (least-significant bit first);
  * MaxCut quality of bitstring j is the (weighted) number of cut edges, or the
    number of uncut edges for the paper's Example 1 form;
  * one numpy Generator per workload; draw order graph -> weights -> gammas -> ts.
"""

from .graphs import (
    ring_edges,
    circular_ladder_edges,
    erdos_renyi_edges,
    random_regular_edges,
)
from .problems import (
    maxcut_qualities,
    maxcut_qualities_device,
    ring_cut_qualities_device,
    portfolio_qualities,
    draw_angles,
    random_symmetric_lambda,
    Workload,
    qaoa_maxcut_workload,
    qwoa_portfolio_workload,
    qwoa_constrained_workload,
    maxcut_zterms,
    exqaoa_maxcut_workload,
    dicke_state,
    dicke_state_device,
    qaoaz_portfolio_workload,
    batched_workloads,
    CONFIG_SEEDS,
)

__all__ = [
    "ring_edges",
    "circular_ladder_edges",
    "erdos_renyi_edges",
    "random_regular_edges",
    "maxcut_qualities",
    "maxcut_qualities_device",
    "ring_cut_qualities_device",
    "portfolio_qualities",
    "draw_angles",
    "random_symmetric_lambda",
    "Workload",
    "qaoa_maxcut_workload",
    "qwoa_portfolio_workload",
    "qwoa_constrained_workload",
    "maxcut_zterms",
    "exqaoa_maxcut_workload",
    "dicke_state",
    "dicke_state_device",
    "qaoaz_portfolio_workload",
    "batched_workloads",
    "CONFIG_SEEDS",
]
