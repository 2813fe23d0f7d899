"""Contraction reference: brute force, the bucket schedule and sliced bucket
elimination in complex128 -- TEST INFRASTRUCTURE (see package header).

Conventions (readings of the paper):

* A tensor over variables (v_0, ..., v_{r-1}) is stored row-major with v_0
  the most significant index; every variable takes the values 0 and 1
  (L = 2, Sec. 2.1).
* Slice s of a deletion set mu = (mu_0, ..., mu_{m-1}) (listed in the order
  Alg. 2 chose them) fixes mu_j to bit j of s (Eq. 3; the paper counts values
  1..L, here 0..L-1).  Fixing keeps the relative order of the other
  variables of each tensor.
* Bucket elimination (Eq. 2, Sec. 2.4): every tensor starts in the bucket of
  its earliest variable in the reduced order; a tensor without variables
  multiplies the slice's scalar.  Buckets are processed in order; the
  bucket of u multiplies its tensors over the union U_b of their variables
  and sums u out.  The result's variables are U_b minus u, sorted by
  position in the order (the paper's index order of intermediates is
  arbitrary); it joins the bucket of its earliest variable, or the scalar.
* A bucket lists its input tensors by id, followed by intermediates in the
  order they were produced.
* The amplitude is the sum of the slice results (Eq. 4), accumulated in
  complex128 with correctly rounded real and imaginary parts.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

LETTERS = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"


# ------------------------------------------------------------- brute force --

def brute_force_sum(n_vars: int, tensors) -> complex:
    """Eq. 1 as a literal sum over every assignment of every variable."""
    if n_vars > 22:
        raise ValueError("brute force is for tiny networks only")
    assign = np.arange(1 << n_vars, dtype=np.int64)
    total = np.ones(1 << n_vars, dtype=np.complex128)
    for vs, data in tensors:
        flat = np.asarray(data, dtype=np.complex128).reshape(-1)
        idx = np.zeros(1 << n_vars, dtype=np.int64)
        r = len(vs)
        for j, v in enumerate(vs):
            idx |= ((assign >> v) & 1) << (r - 1 - j)
        total *= flat[idx]
    return complex(math.fsum(total.real), math.fsum(total.imag))


# ---------------------------------------------------------------- schedule --

@dataclass
class Operand:
    kind: str               # "t": input tensor, "r": intermediate of a step
    ident: int              # tensor id or step index
    vars: Tuple[int, ...]   # variables after fixing sliced ones


@dataclass
class Step:
    var: int                      # the eliminated variable u
    operands: List[Operand]
    union: Tuple[int, ...]        # U_b, sorted by position in the order
    out: Tuple[int, ...]          # U_b minus u, sorted by position


@dataclass
class Schedule:
    order: List[int]              # reduced elimination order
    mu: List[int]                 # sliced variables, bit j of the slice = mu[j]
    steps: List[Step]
    scalar_inputs: List[int]      # input tensors left without variables
    scalar_steps: List[int]       # steps whose result has no variables
    free_vars: List[int]          # order variables appearing in no tensor


def bucket_schedule(n_vars: int, tensor_vars: Sequence[Sequence[int]],
                    order: Sequence[int], mu: Sequence[int]) -> Schedule:
    """The bucket schedule of Eq. 2 for the reduced order and sliced set."""
    sliced = set(mu)
    if sliced & set(order) or len(set(order)) != len(order):
        raise ValueError("order and mu must be disjoint and repetition free")
    if set(order) | sliced != set(range(n_vars)):
        raise ValueError("order + mu must cover every variable")
    pos = {v: i for i, v in enumerate(order)}
    buckets = {v: [] for v in order}
    scalar_inputs = []
    for t, vs in enumerate(tensor_vars):
        rem = tuple(v for v in vs if v not in sliced)
        if not rem:
            scalar_inputs.append(t)
            continue
        buckets[min(rem, key=pos.__getitem__)].append(Operand("t", t, rem))
    steps: List[Step] = []
    scalar_steps: List[int] = []
    free_vars: List[int] = []
    for u in order:
        ops = buckets[u]
        if not ops:
            free_vars.append(u)
            continue
        union = tuple(sorted({v for op in ops for v in op.vars}, key=pos.__getitem__))
        out = tuple(v for v in union if v != u)
        k = len(steps)
        steps.append(Step(u, ops, union, out))
        if out:
            buckets[out[0]].append(Operand("r", k, out))
        else:
            scalar_steps.append(k)
    return Schedule(list(order), list(mu), steps, scalar_inputs, scalar_steps, free_vars)


def schedule_dump(s: Schedule) -> str:
    """Canonical text form of a schedule (compared byte for byte)."""
    lines = ["order " + " ".join(map(str, s.order)),
             "mu " + " ".join(map(str, s.mu)),
             "scalar_inputs " + " ".join(map(str, s.scalar_inputs)),
             "free_vars " + " ".join(map(str, s.free_vars))]
    for k, st in enumerate(s.steps):
        ops = " ".join(f"{o.kind}{o.ident}" for o in st.operands)
        lines.append(f"step {k} var {st.var} ops {ops} union "
                     + " ".join(map(str, st.union)) + " out " + " ".join(map(str, st.out)))
    lines.append("scalar_steps " + " ".join(map(str, s.scalar_steps)))
    return "\n".join(lines) + "\n"


# ------------------------------------------------------ bucket elimination --

def fix_slice(tensors, mu: Sequence[int], s: int):
    """Eq. 3: every tensor with a sliced variable is taken at its fixed value."""
    fixed = {v: (s >> j) & 1 for j, v in enumerate(mu)}
    out = []
    for vs, data in tensors:
        d = np.asarray(data, dtype=np.complex128)
        idx = tuple(fixed[v] if v in fixed else slice(None) for v in vs)
        rem = tuple(v for v in vs if v not in fixed)
        out.append((rem, np.asarray(d[idx], dtype=np.complex128)))
    return out


def contract_slice(tensors, sched: Schedule, s: int) -> complex:
    """sigma_s: bucket elimination of slice s along the schedule (Eq. 2)."""
    fixed = fix_slice(tensors, sched.mu, s)
    scalar = complex(1.0)
    for t in sched.scalar_inputs:
        scalar *= complex(fixed[t][1])
    results = []
    for st in sched.steps:
        letter = {v: LETTERS[i] for i, v in enumerate(st.union)}
        arrays = []
        specs = []
        for op in st.operands:
            if op.kind == "t":
                vs, arr = fixed[op.ident]
            else:
                vs, arr = op.vars, results[op.ident]
            assert tuple(vs) == op.vars
            specs.append("".join(letter[v] for v in vs))
            arrays.append(arr)
        expr = ",".join(specs) + "->" + "".join(letter[v] for v in st.out)
        results.append(np.einsum(expr, *arrays))
    for k in sched.scalar_steps:
        scalar *= complex(results[k])
    scalar *= 2.0 ** len(sched.free_vars)
    return scalar


def exact_sum(values) -> complex:
    vals = [complex(v) for v in values]
    return complex(math.fsum(v.real for v in vals), math.fsum(v.imag for v in vals))


def contract(tensors, sched: Schedule, slices=None):
    """Eq. 4: the sum of sigma_s over the given slices (all by default).

    Returns ``(total, per_slice_values)``.
    """
    m = len(sched.mu)
    if slices is None:
        slices = range(1 << m)
    vals = [contract_slice(tensors, sched, s) for s in slices]
    return exact_sum(vals), vals
