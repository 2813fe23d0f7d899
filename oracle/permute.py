"""Re-ordering the variables of a tensor stored over binary variables
(Sec. 2.1: an intermediate is a tensor over a clique of variables; the same
tensor may be stored in any order of them).

Test infrastructure: used only by the tests.

A tensor over r binary variables is a flat array of 2^r entries whose linear
index has bit p equal to variable p's value (bit 0 the fastest).  Permuting
by ``perm`` moves input bit perm[j] to output bit j:
    out[sum_j x_{perm[j]} 2^j] = in[sum_p x_p 2^p].

* ``permute_bits``: that definition as a numpy axis transpose over the
  [2] * r view (a library primitive standing for the re-indexing).
* ``permute_bits_loop``: the same definition written out entry by entry
  (pure Python, small r only).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def permute_bits(x: np.ndarray, r: int, perm: Sequence[int]) -> np.ndarray:
    """x: [..., 2^r] (any leading batch shape); returns the permuted copy."""
    perm = [int(p) for p in perm]
    assert sorted(perm) == list(range(r))
    lead = x.shape[:-1]
    assert x.shape[-1] == 1 << r
    a = x.reshape(lead + (2,) * r)
    nb = len(lead)
    # In the C-order [2] * r view, axis q holds bit r - 1 - q.  Output axis q
    # holds output bit r - 1 - q, which is input bit perm[r - 1 - q], found at
    # input axis r - 1 - perm[r - 1 - q].
    axes = list(range(nb)) + [nb + r - 1 - perm[r - 1 - q] for q in range(r)]
    return np.ascontiguousarray(a.transpose(axes)).reshape(x.shape)


def permute_bits_loop(x: np.ndarray, r: int, perm: Sequence[int]) -> np.ndarray:
    """Entry-by-entry form for one tensor of 2^r entries."""
    out = np.empty_like(x)
    for i in range(1 << r):
        o = 0
        for j in range(r):
            o |= ((i >> perm[j]) & 1) << j
        out[o] = x[i]
    return out
