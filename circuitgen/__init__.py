"""Seeded synthetic inputs: random grid circuits and their graphical models.

This module only *builds inputs*.  It holds none of the contraction, planning
or cost arithmetic of the method; both the CPU oracle and the GPU library take
what it produces as plain data.

Circuit family (a stand-in for the random-circuit files of Boixo et al. that
the paper's experiments use in Section 4, which are not available here):

* an R x C grid of qubits, qubit ``q = r * C + c``;
* a layer of Hadamards, ``depth`` cycles, and a final layer of Hadamards;
* cycle ``d`` applies CZ to every nearest-neighbour pair of grid pattern
  ``d mod 8`` (eight fixed patterns, every grid edge occurs once per 8 cycles);
* every qubit not touched by a CZ in that cycle gets one of
  {sqrt(X), sqrt(Y), T}, drawn as ``next() % 3`` from a SplitMix64 stream
  (Steele, Lea and Flood, OOPSLA 2014) seeded with the circuit seed;
* the bitstring ``x`` of the amplitude <x|C|0^n> is the next value of the
  same stream, masked to n bits; bit q of x is the value of qubit q.

Graphical model (Section 2.1: variables are the nodes, every tensor is a
clique over its variables):

* every qubit starts on a fresh variable carrying the rank-1 tensor [1, 0];
* a non-diagonal one-qubit gate U opens a new variable; its rank-2 tensor over
  (v_in, v_out) holds U[v_out, v_in];
* a diagonal one-qubit gate (T) is a rank-1 tensor on the current variable;
* CZ is a rank-2 tensor (-1)^(a b) over the two current variables;
* the last variable of qubit q carries the rank-1 tensor e_{x_q}.

Tensor data is complex128, row-major over the tensor's variable list with the
first listed variable the most significant index.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 as published by Steele, Lea and Flood (2014)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)


# ---------------------------------------------------------------- circuits --

def cz_pattern(rows: int, cols: int, p: int) -> List[Tuple[int, int]]:
    """Qubit pairs of CZ pattern p (0..7), sorted.

    Patterns, in order: H(0,0) H(1,1) V(0,0) V(1,1) H(1,0) H(0,1) V(1,0)
    V(0,1), where H(a,b) pairs (r,c)-(r,c+1) with c = a, r = b (mod 2) and
    V(a,b) pairs (r,c)-(r+1,c) with r = a, c = b (mod 2).
    """
    kind, a, b = [("H", 0, 0), ("H", 1, 1), ("V", 0, 0), ("V", 1, 1),
                  ("H", 1, 0), ("H", 0, 1), ("V", 1, 0), ("V", 0, 1)][p % 8]
    pairs = []
    for r in range(rows):
        for c in range(cols):
            if kind == "H":
                if c + 1 < cols and c % 2 == a and r % 2 == b:
                    pairs.append((r * cols + c, r * cols + c + 1))
            else:
                if r + 1 < rows and r % 2 == a and c % 2 == b:
                    pairs.append((r * cols + c, (r + 1) * cols + c))
    return sorted(pairs)


ONE_QUBIT_DRAW = ("sqrtX", "sqrtY", "T")


@dataclass
class Circuit:
    rows: int
    cols: int
    depth: int
    seed: int
    gates: List[tuple] = field(default_factory=list)  # ("H", q) / ("CZ", a, b) ...
    bitstring: int = 0

    @property
    def n_qubits(self) -> int:
        return self.rows * self.cols


def random_grid_circuit(rows: int, cols: int, depth: int, seed: int) -> Circuit:
    """Seeded random grid circuit of the family described in the module doc."""
    n = rows * cols
    rng = SplitMix64(seed)
    gates: List[tuple] = [("H", q) for q in range(n)]
    for d in range(depth):
        pairs = cz_pattern(rows, cols, d)
        hit = set()
        for a, b in pairs:
            gates.append(("CZ", a, b))
            hit.add(a)
            hit.add(b)
        for q in range(n):
            if q not in hit:
                gates.append((ONE_QUBIT_DRAW[rng.next() % 3], q))
    gates += [("H", q) for q in range(n)]
    x = rng.next() & ((1 << n) - 1)
    return Circuit(rows, cols, depth, seed, gates, x)


# ------------------------------------------------------------------ models --

_S2 = 1.0 / np.sqrt(2.0)
# Gate matrices, indexed [out, in].
GATE_MATRIX = {
    "H": np.array([[_S2, _S2], [_S2, -_S2]], dtype=np.complex128),
    "sqrtX": 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128),
    "sqrtY": 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128),
}
T_DIAG = np.array([1.0, np.exp(1j * np.pi / 4)], dtype=np.complex128)
CZ_TENSOR = np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128)


@dataclass
class Model:
    """A graphical model: ``n_vars`` binary variables and a list of tensors.

    ``tensors[t] = (vars, data)`` with ``data.shape == (2,) * len(vars)``.
    """
    n_vars: int
    tensors: List[Tuple[Tuple[int, ...], np.ndarray]]

    def flat(self):
        """(rank int32[T], vars int32[sum rank], data float64[2 * sum 2^rank])."""
        rank = np.array([len(v) for v, _ in self.tensors], dtype=np.int32)
        vars_ = np.array([x for v, _ in self.tensors for x in v], dtype=np.int32)
        parts = [np.ascontiguousarray(d, dtype=np.complex128).reshape(-1) for _, d in self.tensors]
        data = np.concatenate(parts).view(np.float64) if parts else np.zeros(0)
        return rank, vars_, np.ascontiguousarray(data)


def circuit_model(circ: Circuit, bitstring: int | None = None) -> Model:
    """Graphical model of <x|C|0^n> (construction in the module doc)."""
    x = circ.bitstring if bitstring is None else bitstring
    n = circ.n_qubits
    tensors: List[Tuple[Tuple[int, ...], np.ndarray]] = []
    cur = list(range(n))
    nv = n
    for q in range(n):
        tensors.append(((q,), np.array([1.0, 0.0], dtype=np.complex128)))
    for g in circ.gates:
        name = g[0]
        if name == "CZ":
            a, b = g[1], g[2]
            tensors.append(((cur[a], cur[b]), CZ_TENSOR.copy()))
        elif name == "T":
            q = g[1]
            tensors.append(((cur[q],), T_DIAG.copy()))
        else:
            q = g[1]
            u = GATE_MATRIX[name]
            tensors.append(((cur[q], nv), u.T.copy()))  # data[v_in, v_out] = U[v_out, v_in]
            cur[q] = nv
            nv += 1
    for q in range(n):
        bit = (x >> q) & 1
        e = np.zeros(2, dtype=np.complex128)
        e[bit] = 1.0
        tensors.append(((cur[q],), e))
    return Model(nv, tensors)


def model_from_flat(n_vars: int, rank: Sequence[int], vars_: Sequence[int], data: np.ndarray) -> Model:
    tensors = []
    vp = 0
    dp = 0
    data = np.asarray(data, dtype=np.float64)
    for r in rank:
        vs = tuple(int(v) for v in vars_[vp:vp + r])
        size = 1 << r
        d = data[2 * dp:2 * (dp + size)].view(np.complex128).reshape((2,) * r).copy()
        tensors.append((vs, d))
        vp += r
        dp += size
    return Model(n_vars, tensors)


# --------------------------------------------------------- toy networks ----

def toy_network(seed: int = 0) -> Model:
    """The seven-tensor network of Eq. (1) with seeded random complex entries.

    Variable ids: i=0 j=1 k=2 l=3 m=4 n=5.  Tensors, in order:
    A_i B_ijk C_jl D_kl E_km F_ln G_mn.
    """
    rng = np.random.default_rng(seed)
    spec = [(0,), (0, 1, 2), (1, 3), (2, 3), (2, 4), (3, 5), (4, 5)]
    tensors = []
    for vs in spec:
        shape = (2,) * len(vs)
        d = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        tensors.append((vs, d.astype(np.complex128)))
    return Model(6, tensors)


TOY_NAMES = "ijklmn"


def random_network(n_vars: int, n_tensors: int, max_rank: int, seed: int) -> Model:
    """Seeded random binary tensor network (every variable appears at least once)."""
    rng = np.random.default_rng(seed)
    tensors = []
    for t in range(n_tensors):
        r = int(rng.integers(1, max_rank + 1))
        vs = tuple(int(v) for v in rng.choice(n_vars, size=min(r, n_vars), replace=False))
        shape = (2,) * len(vs)
        d = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        tensors.append((vs, d.astype(np.complex128)))
    seen = {v for vs, _ in tensors for v in vs}
    for v in range(n_vars):
        if v not in seen:
            d = rng.standard_normal(2) + 1j * rng.standard_normal(2)
            tensors.append(((v,), d.astype(np.complex128)))
    return Model(n_vars, tensors)


# ----------------------------------------------------- workload recipes ----

# Named workloads (grid rows, cols, depth, sliced variables m).
WORKLOADS = {
    "grid4x4_d10_m0": (4, 4, 10, 0),
    "grid5x5_d16_m6": (5, 5, 16, 6),
    "grid7x7_d24_m10": (7, 7, 24, 10),
}


def batch_instances(count: int = 512, first_seed: int = 1000):
    """Uneven instance mix: rows, cols uniform in {4,5,6}; depth uniform in
    {10..20}; sliced variables m uniform in {0..6}; one bitstring each.

    Returns a list of (rows, cols, depth, m, seed).
    """
    out = []
    for i in range(count):
        seed = first_seed + i
        rng = SplitMix64(seed ^ 0xA5A5A5A5A5A5A5A5)
        r = 4 + rng.next() % 3
        c = 4 + rng.next() % 3
        d = 10 + rng.next() % 11
        m = rng.next() % 7
        out.append((int(r), int(c), int(d), int(m), seed))
    return out


def random_general_network(seed: int, n_vars: int = 7, n_tensors: int = 7, max_rank: int = 3,
                           max_dim: int = 5):
    """A random network over variables of dimensions 1..max_dim (numpy
    default_rng(seed)): returns (dims, tensors), tensors as (vars, data)
    with data shaped by the variables' dimensions; every variable occurs in
    some tensor."""
    rng = np.random.default_rng(seed)
    dims = [int(rng.integers(1, max_dim + 1)) for _ in range(n_vars)]
    tensors = []
    for _ in range(n_tensors):
        r = int(rng.integers(1, max_rank + 1))
        vs = tuple(int(v) for v in rng.choice(n_vars, size=r, replace=False))
        shape = [dims[v] for v in vs]
        tensors.append((vs, rng.standard_normal(shape) + 1j * rng.standard_normal(shape)))
    for v in range(n_vars):
        if not any(v in vs for vs, _ in tensors):
            tensors.append(((v,), rng.standard_normal(dims[v]) + 1j * rng.standard_normal(dims[v])))
    return dims, tensors


def star_network(n_leaves: int, seed: int, max_phase: float = 0.3) -> Model:
    """A hub variable 0 joined to leaves 1..n_leaves by one rank-2 tensor
    each, T_i over (0, i).  Entries are (0.5 + 0.5 u) e^(i phi) with u,
    phi / max_phase uniform in [0, 1) (numpy default_rng(seed)): no sum
    cancels.  Eliminating the hub first makes one intermediate over all
    leaves (rank n_leaves), the largest a network of this size can hold."""
    rng = np.random.default_rng(seed)
    tensors = []
    for i in range(1, n_leaves + 1):
        mag = 0.5 + 0.5 * rng.random((2, 2))
        phase = max_phase * rng.random((2, 2))
        tensors.append(((0, i), (mag * np.exp(1j * phase)).astype(np.complex128)))
    return Model(n_leaves + 1, tensors)
