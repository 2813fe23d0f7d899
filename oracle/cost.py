"""Cost model of a bucket schedule -- TEST INFRASTRUCTURE (see package header).

Sec. 4 states that per-subtask memory grows as 2^tau and FLOPs as
2^(tau+1), and that the total over all subtasks is 2^|mu| times the
per-subtask count; the exact formulas it defers to another paper, so the
following are this project's, in the exponents of Eq. 2 (step cost L^|U_b|):

* bucket b with k operands over the union U_b, result rank r_b = |U_b| - 1:
  FLOPs_b = 6 (k - 1) 2^|U_b| + 2 * 2^r_b real flops (k - 1 complex
  products over U_b, then one complex addition per result entry for the
  sum over u; the first term vanishes for k = 1);
* algorithmic bytes_b = 8 (sum_i 2^rank(T_i) + 2^r_b) in complex64;
* peak memory = the largest, over the steps, of the bytes held by tensors
  not yet consumed (inputs and intermediates, operands of the current step
  included) plus the current step's result; tensors without variables are
  scalars and hold nothing;
* the totals for all slices are 2^m times the per-slice figures.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

from .contract import Schedule


@dataclass
class StepCost:
    flops: int
    bytes: int


@dataclass
class Cost:
    steps: List[StepCost]
    flops_per_slice: int
    bytes_per_slice: int
    peak_bytes: int
    width: int           # largest |U_b| - 1 over the steps
    n_slices: int

    @property
    def total_flops(self) -> int:
        return self.flops_per_slice * self.n_slices

    @property
    def total_bytes(self) -> int:
        return self.bytes_per_slice * self.n_slices


def schedule_cost(sched: Schedule, elem_bytes: int = 8) -> Cost:
    steps = []
    for st in sched.steps:
        k = len(st.operands)
        nu = len(st.union)
        flops = (6 * (k - 1) * (1 << nu) if k > 1 else 0) + 2 * (1 << (nu - 1))
        byts = elem_bytes * (sum(1 << len(op.vars) for op in st.operands) + (1 << (nu - 1)))
        steps.append(StepCost(flops, byts))

    # peak live memory
    live = {}
    for st in sched.steps:
        for op in st.operands:
            if op.kind == "t":
                live[("t", op.ident)] = elem_bytes * (1 << len(op.vars))
    peak = 0
    for k, st in enumerate(sched.steps):
        out_bytes = elem_bytes * (1 << len(st.out)) if st.out else 0
        peak = max(peak, sum(live.values()) + out_bytes)
        for op in st.operands:
            live.pop((op.kind, op.ident), None)
        if st.out:
            live[("r", k)] = out_bytes
    width = max((len(st.union) - 1 for st in sched.steps), default=0)
    return Cost(steps, sum(s.flops for s in steps), sum(s.bytes for s in steps),
                peak, width, 1 << len(sched.mu))
