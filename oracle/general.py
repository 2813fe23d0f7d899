"""Networks over variables of any dimension L (Sec. 2.1 states the
contraction for general L; the quantum-circuit workloads have L = 2).

Test infrastructure: used only by the tests.  complex128 throughout.

* ``contract_general``: the plain definition -- the sum over all joint
  assignments of the product of the tensors -- as one numpy einsum (a
  library primitive standing for that sum; no order or slicing involved).
* ``binary_expansion``: the equivalent network over binary variables: a
  variable of dimension L becomes ceil(log2 L) binary variables (its index
  bits, most significant first), tensors are re-laid out over those bits,
  and index values >= L get entry 0.  Sums over the expansion equal sums
  over the original because the padded values contribute zero.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

Tensor = Tuple[Tuple[int, ...], np.ndarray]


def contract_general(dims: Sequence[int], tensors: Sequence[Tensor]) -> complex:
    """Sum over every assignment of every variable of the product."""
    letters = {}
    operands = []
    for vs, data in tensors:
        d = np.asarray(data, dtype=np.complex128).reshape([dims[v] for v in vs])
        sub = []
        for v in vs:
            if v not in letters:
                letters[v] = len(letters)
            sub.append(letters[v])
        operands += [d, sub]
    if not operands:
        return complex(np.prod([float(x) for x in dims]))
    total = complex(np.einsum(*operands, []))
    # variables in no tensor multiply the sum by their dimension
    for v, L in enumerate(dims):
        if v not in letters:
            total *= L
    return total


def binary_expansion(dims: Sequence[int], tensors: Sequence[Tensor]):
    """Returns (n_binary_vars, binary tensors, first, count) with first[v],
    count[v] the binary variables of variable v."""
    first, count = [], []
    n = 0
    for L in dims:
        b = 0
        while (1 << b) < L:
            b += 1
        first.append(n)
        count.append(b)
        n += b
    out: List[Tensor] = []
    for vs, data in tensors:
        d = np.asarray(data, dtype=np.complex128).reshape([dims[v] for v in vs])
        bvars = tuple(first[v] + k for v in vs for k in range(count[v]))
        padded = np.zeros([1 << count[v] for v in vs], dtype=np.complex128)
        padded[tuple(slice(0, dims[v]) for v in vs)] = d
        out.append((bvars, padded.reshape((2,) * len(bvars)) if bvars else padded.reshape(())))
    return n, out, first, count
