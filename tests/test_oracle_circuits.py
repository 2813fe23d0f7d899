"""Pins of the oracle on quantum circuits: statevector simulation (the plain
definition of <x|C|0^n>), the unit norm of the output state, textbook gate
identities and the depth-0 circuit (H H = I)."""
import json
import os

import numpy as np
import pytest

from circuitgen import (WORKLOADS, circuit_model, cz_pattern, random_grid_circuit)
from oracle import contract as C
from oracle import planner as P
from oracle import statevector as SV

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def oracle_amplitude(circ, m=0, bitstring=None):
    mod = circuit_model(circ, bitstring)
    tv = [v for v, _ in mod.tensors]
    adj = P.simple_graph(mod.n_vars, tv)
    order = P.min_fill_order(adj)
    mu, _, pi, _ = P.greedy_treewidth_deletion(adj, order, m)
    total, _ = C.contract(mod.tensors, C.bucket_schedule(mod.n_vars, tv, pi, mu))
    return total


def test_gate_identities():
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
    M = SV.MATRICES
    for g in M.values():
        assert np.allclose(g.conj().T @ g, np.eye(2), atol=1e-15)
    assert np.allclose(M["sqrtX"] @ M["sqrtX"], X, atol=1e-15)
    assert np.allclose(M["sqrtY"] @ M["sqrtY"], Y, atol=1e-15)
    assert np.allclose(M["H"] @ M["H"], np.eye(2), atol=1e-15)
    T8 = np.linalg.matrix_power(M["T"], 8)
    assert np.allclose(T8, np.eye(2), atol=1e-14)


def test_cz_patterns_cover_each_edge_once_per_8_cycles():
    for rows, cols in [(4, 4), (5, 5), (3, 6), (7, 7)]:
        seen = []
        for p in range(8):
            used = set()
            for a, b in cz_pattern(rows, cols, p):
                assert a not in used and b not in used  # a pattern is a matching
                used |= {a, b}
                seen.append((a, b))
        n_edges = rows * (cols - 1) + (rows - 1) * cols
        assert len(seen) == n_edges == len(set(seen))


@pytest.mark.parametrize("rows,cols,depth,seed", [(2, 2, 3, 0), (2, 3, 5, 1), (3, 3, 6, 2),
                                                  (3, 3, 8, 3), (3, 4, 8, 4), (4, 4, 10, 0)])
def test_oracle_matches_statevector(rows, cols, depth, seed):
    circ = random_grid_circuit(rows, cols, depth, seed)
    n = rows * cols
    psi = SV.statevector(n, circ.gates)
    rng = np.random.default_rng(seed)
    xs = [circ.bitstring] + [int(x) for x in rng.integers(0, 1 << n, size=3)]
    for x in xs:
        got = oracle_amplitude(circ, m=min(2, n), bitstring=x)
        assert abs(got - psi[x]) <= 1e-12, (x, got, psi[x])


@pytest.mark.parametrize("rows,cols,depth,seed", [(2, 3, 6, 5), (3, 3, 5, 7)])
def test_unit_norm_over_all_bitstrings(rows, cols, depth, seed):
    circ = random_grid_circuit(rows, cols, depth, seed)
    n = rows * cols
    total = sum(abs(oracle_amplitude(circ, m=1, bitstring=x)) ** 2 for x in range(1 << n))
    assert abs(total - 1.0) <= 1e-12


@pytest.mark.parametrize("rows,cols", [(2, 2), (3, 3)])
def test_depth_zero_is_identity(rows, cols):
    circ = random_grid_circuit(rows, cols, 0, 0)
    n = rows * cols
    for x in range(1 << n):
        want = 1.0 if x == 0 else 0.0
        assert abs(oracle_amplitude(circ, bitstring=x) - want) <= 1e-13


def test_golden_amplitudes_match_oracle():
    """Stored statevector amplitudes (written by tests/golden/make_golden.py,
    which calls only the oracle) against the oracle's sliced contraction."""
    gold = json.load(open(os.path.join(GOLD, "amplitudes.json")))
    for name in ("grid4x4_d10_m0", "grid5x5_d16_m6"):
        g = gold[name]
        rows, cols, depth, m = WORKLOADS[name]
        circ = random_grid_circuit(rows, cols, depth, g["seed"])
        assert circ.bitstring == g["bitstring"]
        sv = complex(*g["statevector"])
        got = oracle_amplitude(circ, m=m)
        assert abs(got - sv) <= 1e-12
        # benchmark seeds are chosen with a non-degenerate amplitude
        assert (1 << (rows * cols)) * abs(sv) ** 2 >= 1e-2


def test_golden_7x7_slices_match_oracle():
    gold = json.load(open(os.path.join(GOLD, "amplitudes.json")))["grid7x7_d24_m10"]
    rows, cols, depth, m = WORKLOADS["grid7x7_d24_m10"]
    circ = random_grid_circuit(rows, cols, depth, gold["seed"])
    mod = circuit_model(circ)
    tv = [v for v, _ in mod.tensors]
    adj = P.simple_graph(mod.n_vars, tv)
    order = P.min_fill_order(adj)
    mu, _, pi, tau = P.greedy_treewidth_deletion(adj, order, m)
    assert tau == gold["tau"] and tau <= 28
    sched = C.bucket_schedule(mod.n_vars, tv, pi, mu)
    for s in (0, 5):
        got = C.contract_slice(mod.tensors, sched, s)
        want = complex(*gold["slices"][s])
        assert abs(got - want) <= 1e-13 * max(abs(want), 1e-30) + 1e-30
