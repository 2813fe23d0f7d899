"""Dense statevector simulation -- the plain definition of <x|C|0^n>.

Test infrastructure (see the package header).  The gate matrices are written
here independently of the model builder, so that a wrong matrix on either
side shows up as a mismatch.  Basis index convention: bit q of the index is
the value of qubit q.
"""
from __future__ import annotations

import numpy as np

_R = 1.0 / np.sqrt(2.0)
# Textbook one-qubit gates, [row = output, column = input].
MATRICES = {
    "H": np.array([[_R, _R], [_R, -_R]], dtype=np.complex128),
    "sqrtX": np.array([[0.5 + 0.5j, 0.5 - 0.5j], [0.5 - 0.5j, 0.5 + 0.5j]], dtype=np.complex128),
    "sqrtY": np.array([[0.5 + 0.5j, -0.5 - 0.5j], [0.5 + 0.5j, 0.5 + 0.5j]], dtype=np.complex128),
    "T": np.array([[1.0, 0.0], [0.0, np.cos(np.pi / 4) + 1j * np.sin(np.pi / 4)]], dtype=np.complex128),
}


def _axis(n: int, q: int) -> int:
    # C-order reshape to (2,)*n puts the least significant bit on the last axis.
    return n - 1 - q


def apply_gate(psi: np.ndarray, n: int, gate: tuple) -> None:
    """Apply one gate in place to a 2^n statevector."""
    t = psi.reshape((2,) * n)
    if gate[0] == "CZ":
        ia, ib = _axis(n, gate[1]), _axis(n, gate[2])
        sl = [slice(None)] * n
        sl[ia] = 1
        sl[ib] = 1
        t[tuple(sl)] *= -1.0
        return
    u = MATRICES[gate[0]]
    ax = _axis(n, gate[1])
    s0 = [slice(None)] * n
    s1 = [slice(None)] * n
    s0[ax] = 0
    s1[ax] = 1
    a = t[tuple(s0)].copy()
    b = t[tuple(s1)].copy()
    t[tuple(s0)] = u[0, 0] * a + u[0, 1] * b
    t[tuple(s1)] = u[1, 0] * a + u[1, 1] * b


def statevector(n: int, gates) -> np.ndarray:
    """C|0^n> as a complex128 vector of length 2^n."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    for g in gates:
        apply_gate(psi, n, g)
    return psi


def amplitude(n: int, gates, x: int) -> complex:
    """<x|C|0^n> by full statevector simulation."""
    return complex(statevector(n, gates)[x])
