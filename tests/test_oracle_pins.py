"""Pins of the CPU oracle against the paper's worked example and hand counts.

Every expectation here comes from the paper (Eq. 1-3, Figs. 3, 4, 6 and the
text of Secs. 2-3) or from a hand derivation recorded in
``tests/golden/toy_figures.json``; none is produced by the code under test.
"""
import json
import os

import numpy as np
import pytest

from circuitgen import random_general_network, toy_network
from oracle import contract as C
from oracle import cost as K
from oracle import planner as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FIG = json.load(open(os.path.join(GOLD, "toy_figures.json")))
PI = [0, 1, 2, 3, 4, 5]  # [i j k l m n]


def toy_graph():
    m = toy_network(0)
    return P.simple_graph(6, [v for v, _ in m.tensors])


def test_toy_graph_edges_match_eq1():
    adj = toy_graph()
    edges = sorted((a, b) for a in adj for b in adj[a] if a < b)
    assert edges == [tuple(e) for e in FIG["edges"]]


def test_eq2_schedule_is_the_worked_example():
    m = toy_network(0)
    s = C.bucket_schedule(6, [v for v, _ in m.tensors], PI, [])
    want = "".join(l for l in open(os.path.join(GOLD, "toy_eq2_schedule.txt")).readlines()
                   if not l.startswith("#"))
    assert C.schedule_dump(s) == want


def test_eq2_step_cost_exponents():
    m = toy_network(0)
    s = C.bucket_schedule(6, [v for v, _ in m.tensors], PI, [])
    assert [len(st.union) for st in s.steps] == FIG["eq2_cost_exponents"]


@pytest.mark.parametrize("seed", range(5))
def test_bucket_elimination_equals_brute_force_on_toy(seed):
    m = toy_network(seed)
    s = C.bucket_schedule(6, [v for v, _ in m.tensors], PI, [])
    got, _ = C.contract(m.tensors, s)
    want = C.brute_force_sum(6, m.tensors)
    assert abs(got - want) <= 1e-12 * max(1.0, abs(want))


def test_alg1_width_fig6():
    assert P.treewidth_from_order(toy_graph(), PI) == FIG["fig6_width_of_order_ijklmn"]


def test_alg4_tree_fig6_and_fig3():
    adj = toy_graph()
    bags, parent = P.clique_tree(adj, PI)
    assert [sorted(b) for b in bags] == FIG["fig6_bags"]
    assert P.td_width(bags) == 2
    assert P.is_valid_td(adj, bags, parent)
    # a path graph: exactly one root, every other bag has one parent
    assert parent.count(-1) == 1
    rbags, rparent = P.clique_tree(adj, FIG["fig3_reverse_order"])
    assert sorted(sorted(b) for b in rbags) == sorted(FIG["fig6_bags"])
    assert P.is_valid_td(adj, rbags, rparent)


def test_fig4_removal_treewidths_by_brute_force():
    adj = toy_graph()
    for u, tw in FIG["fig4_removed_tw"].items():
        assert P.optimal_treewidth(P.remove_vertex(adj, int(u))) == tw


def test_tree_trimming_picks_k_on_toy():
    assert P.tree_trimming_pick(toy_graph(), PI) == FIG["tree_trimming_pick"]


def test_alg2_on_toy_removes_k_and_reaches_width_1():
    mu, g, pi, tau = P.greedy_treewidth_deletion(toy_graph(), PI, 1)
    assert mu == [2]
    assert pi == [0, 1, 3, 4, 5]
    assert tau == 1
    assert 2 not in g and all(2 not in ns for ns in g.values())


def test_alg2_target_width_mode():
    mu, _, _, tau = P.greedy_treewidth_deletion(toy_graph(), PI, -1, target_width=1)
    assert mu == [2] and tau == 1


def test_tree_trimming_uses_union_of_max_bags():
    # Bags {0,1,2} {2,3} {3,4,5} {3,6}: both 3-bags are maximal, so b_max is
    # their union; vertex 3 lies in 3 bags and wins.  Looking at the first
    # maximal bag alone would give 2.
    edges = [(0, 1), (0, 2), (1, 2), (2, 3), (3, 4), (3, 5), (4, 5), (3, 6)]
    adj = {v: set() for v in range(7)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    order = [0, 1, 2, 4, 5, 6, 3]
    bags, parent = P.clique_tree(adj, order)
    assert sorted(sorted(b) for b in bags) == [[0, 1, 2], [2, 3], [3, 4, 5], [3, 6]]
    assert P.is_valid_td(adj, bags, parent)
    assert P.tree_trimming_pick(adj, order) == 3


def test_tree_trimming_length_before_weight():
    # Bags X = {A,B,p,q,r}, Y = {B,s,t,w,z}, {a1,A}, {a2,A}.  A: length 3,
    # weight 9; B: length 2, weight 10.  Length decides first, so A.
    A, B, p, q, r, s, t, w, z, a1, a2 = range(11)
    adj = {v: set() for v in range(11)}

    def clique(vs):
        for x in vs:
            for y in vs:
                if x != y:
                    adj[x].add(y)
    clique([A, B, p, q, r])
    clique([B, s, t, w, z])
    clique([A, a1])
    clique([A, a2])
    order = [a1, a2, p, q, r, s, t, w, z, A, B]
    bags, parent = P.clique_tree(adj, order)
    assert sorted(sorted(b) for b in bags) == sorted(
        [sorted([A, B, p, q, r]), sorted([B, s, t, w, z]), [A, a1], [A, a2]])
    assert P.is_valid_td(adj, bags, parent)
    assert P.tree_trimming_pick(adj, order) == A


def test_min_fill_on_toy_by_hand():
    assert P.min_fill_order(toy_graph()) == FIG["min_fill_order"]


def test_min_fill_degree_tie_break():
    # triangle 0-1-2 with a pendant 3 on 0: 1, 2 and 3 have fill 0; 3 has the
    # smallest degree and goes first despite the largest id; then 0, 1, 2.
    adj = {0: {1, 2, 3}, 1: {0, 2}, 2: {0, 1}, 3: {0}}
    assert P.min_fill_order(adj) == [3, 0, 1, 2]


def test_alg1_star_center_first_drops_by_more_than_one():
    # Sec. 3.1's bound of one per removal holds for optimal treewidth; with a
    # fixed order the width can drop by more.
    adj = {0: {1, 2, 3, 4}, 1: {0}, 2: {0}, 3: {0}, 4: {0}}
    assert P.treewidth_from_order(adj, [0, 1, 2, 3, 4]) == 4
    assert P.treewidth_from_order(P.remove_vertex(adj, 0), [1, 2, 3, 4]) == 0
    assert P.optimal_treewidth(adj) == 1


def test_cost_model_hand_count_on_toy():
    m = toy_network(0)
    s = C.bucket_schedule(6, [v for v, _ in m.tensors], PI, [])
    c = K.schedule_cost(s)
    assert [x.flops for x in c.steps] == FIG["flops"]
    assert [x.bytes for x in c.steps] == FIG["bytes"]
    assert c.peak_bytes == FIG["peak_bytes"]
    assert c.width == 2
    assert c.n_slices == 1


def test_cost_totals_scale_with_slices():
    # Sec. 4: total work is 2^|mu| times the per-subtask work.
    m = toy_network(0)
    order = [0, 1, 3, 4, 5]
    s = C.bucket_schedule(6, [v for v, _ in m.tensors], order, [2])
    c = K.schedule_cost(s)
    assert c.n_slices == 2
    assert c.total_flops == 2 * c.flops_per_slice
    assert c.width == 1


def test_slices_fix_k_as_in_eq3():
    # sigma_v is the brute-force sum restricted to k = v (Eq. 3); the two add
    # up to sigma (Eq. 4).
    m = toy_network(3)
    order = [0, 1, 3, 4, 5]
    s = C.bucket_schedule(6, [v for v, _ in m.tensors], order, [2])
    total, vals = C.contract(m.tensors, s)
    for v in (0, 1):
        restricted = []
        for vs, d in m.tensors:
            if 2 in vs:
                mask = np.zeros((2,) * len(vs))
                idx = [slice(None)] * len(vs)
                idx[vs.index(2)] = v
                mask[tuple(idx)] = 1.0
                d = d * mask
            restricted.append((vs, d))
        want = C.brute_force_sum(6, restricted)
        assert abs(vals[v] - want) <= 1e-12 * max(1.0, abs(want))
    full = C.brute_force_sum(6, m.tensors)
    assert abs(total - full) <= 1e-12 * max(1.0, abs(full))


def test_slice_bit_j_fixes_mu_j():
    # Two sliced variables in a chosen order: slice s = 1 sets mu[0] = 1 and
    # mu[1] = 0 (bit j of s fixes mu[j]).
    m = toy_network(4)
    mu = [3, 1]
    order = [0, 2, 4, 5]
    s = C.bucket_schedule(6, [v for v, _ in m.tensors], order, mu)
    _, vals = C.contract(m.tensors, s)
    for sl in range(4):
        want_fix = {3: sl & 1, 1: (sl >> 1) & 1}
        restricted = []
        for vs, d in m.tensors:
            mask = np.ones((2,) * len(vs))
            for var, val in want_fix.items():
                if var in vs:
                    idx = [slice(None)] * len(vs)
                    idx[vs.index(var)] = 1 - val
                    mask[tuple(idx)] = 0.0
            restricted.append((vs, d * mask))
        want = C.brute_force_sum(6, restricted)
        assert abs(vals[sl] - want) <= 1e-12 * max(1.0, abs(want))


def test_free_variable_contributes_factor_two():
    # A variable in no tensor is summed over its L = 2 values.
    t = [((0,), np.array([1.0 + 1j, 2.0]))]
    s = C.bucket_schedule(2, [v for v, _ in t], [0, 1], [])
    got, _ = C.contract(t, s)
    assert abs(got - 2 * (3.0 + 1j)) < 1e-14
    assert abs(C.brute_force_sum(2, t) - got) < 1e-14


def _brute_betweenness(adj):
    """Betweenness by enumerating every shortest path of every unordered
    pair (tiny graphs only): the share of s-t shortest paths through v."""
    import itertools
    from collections import deque
    verts = sorted(adj)

    def dist_from(s):
        d = {s: 0}
        q = deque([s])
        while q:
            v = q.popleft()
            for w in adj[v]:
                if w not in d:
                    d[w] = d[v] + 1
                    q.append(w)
        return d

    dist = {s: dist_from(s) for s in verts}

    def paths(s, t):
        if s == t:
            return [[s]]
        out = []
        for w in adj[s]:
            if w in dist[t] and dist[t][w] == dist[t][s] - 1:
                out += [[s] + p for p in paths(w, t)]
        return out

    bc = {v: 0.0 for v in verts}
    for s, t in itertools.combinations(verts, 2):
        if t not in dist[s]:
            continue
        ps = paths(s, t)
        for v in verts:
            if v not in (s, t):
                bc[v] += sum(v in p for p in ps) / len(ps)
    return bc


def test_betweenness_closed_forms_and_brute_force():
    """Sec. 3.1 betweenness score: on a path of n vertices vertex i lies on
    i (n - 1 - i) shortest paths, so the middle vertex is picked; a star's
    centre lies on all C(n - 1, 2) leaf pairs; on small random graphs the
    pick is the vertex of largest brute-force betweenness (earliest in the
    order on ties)."""
    n = 7
    path = {i: {j for j in (i - 1, i + 1) if 0 <= j < n} for i in range(n)}
    assert P.betweenness_pick(path, list(range(n))) == 3
    bc = _brute_betweenness(path)
    assert all(abs(bc[i] - i * (n - 1 - i)) < 1e-12 for i in range(n))
    star = {0: set(range(1, 6)), **{i: {0} for i in range(1, 6)}}
    assert P.betweenness_pick(star, [3, 1, 0, 2, 4, 5]) == 0
    assert _brute_betweenness(star)[0] == 10
    rng = np.random.default_rng(5)
    for _ in range(20):
        k = int(rng.integers(5, 9))
        adj = {v: set() for v in range(k)}
        for a in range(k):
            for b in range(a + 1, k):
                if rng.random() < 0.35:
                    adj[a].add(b)
                    adj[b].add(a)
        order = [int(v) for v in rng.permutation(k)]
        bc = _brute_betweenness(adj)
        pos = {u: i for i, u in enumerate(order)}
        want = max(adj, key=lambda u: (round(bc[u], 9), -pos[u]))
        assert P.betweenness_pick(adj, order) == want


def test_alg5_recovers_orders_from_tree_decompositions():
    """App. B, Alg. 5: on Fig. 6's chain of bags {ijk}-{jkl}-{klm}-{lmn} the
    leaf-first order has width 2; on random graphs the order recovered from
    the clique tree of an order lists every vertex once and is no wider than
    the decomposition (largest bag minus one)."""
    i, j, k, l, m, n = range(6)
    bags = [frozenset({i, j, k}), frozenset({j, k, l}), frozenset({k, l, m}), frozenset({l, m, n})]
    parent = [1, 2, 3, -1]  # rooted at {lmn}
    order = P.recover_order(bags, parent)
    assert order == [i, j, k, l, m, n]
    adj = {v: set() for v in range(6)}
    for b in bags:
        for a in b:
            adj[a] |= set(b) - {a}
    assert P.treewidth_from_order(adj, order) == 2
    rng = np.random.default_rng(11)
    for _ in range(30):
        nv = int(rng.integers(4, 12))
        adj = {v: set() for v in range(nv)}
        for a in range(nv):
            for b in range(a + 1, nv):
                if rng.random() < 0.3:
                    adj[a].add(b)
                    adj[b].add(a)
        o = [int(v) for v in rng.permutation(nv)]
        bags, parent = P.clique_tree(adj, o)
        rec = P.recover_order(bags, parent)
        assert sorted(rec) == list(range(nv))
        assert P.treewidth_from_order(adj, rec) <= P.td_width(bags)


def test_anytime_order_and_recomputation_reduce_to_the_plain_forms():
    """One try of the anytime heuristic is min-fill, more tries are never
    wider; Alg. 2 without recomputation is the plain greedy deletion, and
    recomputation never widens the final reduced order on these circuits."""
    from circuitgen import circuit_model, random_grid_circuit
    for seed in range(3):
        mod = circuit_model(random_grid_circuit(4, 4, 10, seed))
        adj = P.simple_graph(mod.n_vars, [v for v, _ in mod.tensors])
        o = P.min_fill_order(adj)
        assert P.anytime_order(adj, 1, 5) == o
        assert P.treewidth_from_order(adj, P.anytime_order(adj, 6, 5)) <= P.treewidth_from_order(adj, o)
        plain = P.greedy_treewidth_deletion(adj, o, 3)
        same = P.greedy_treewidth_deletion_recompute(adj, o, 3, 0, 4, 1)
        assert plain[0] == same[0] and plain[2] == same[2] and plain[3] == same[3]
        rec = P.greedy_treewidth_deletion_recompute(adj, o, 3, 1, 4, 1)
        assert rec[3] <= plain[3]


def test_general_dimension_contraction_pins():
    """Sec. 2.1 for general L: an all-ones network sums to the product of
    the dimensions; with L = 2 the definition is the binary brute force; the
    binary expansion (index bits, padded entries 0) has the same sum."""
    from oracle import general as Gn
    dims = [3, 1, 4, 5]
    tensors = [((0, 1), np.ones((3, 1))), ((2, 3), np.ones((4, 5))), ((0, 3), np.ones((3, 5)))]
    # each variable is summed over its L values; variables 0 and 3 are shared
    assert abs(Gn.contract_general(dims, tensors) - 3 * 1 * 4 * 5) < 1e-12
    n, tens = toy_network(seed=2).n_vars, toy_network(seed=2).tensors
    assert abs(Gn.contract_general([2] * n, tens) - C.brute_force_sum(n, tens)) < 1e-9 * abs(C.brute_force_sum(n, tens))
    for seed in range(12):
        dims, tensors = random_general_network(seed)
        want = Gn.contract_general(dims, tensors)
        nb, btens, first, count = Gn.binary_expansion(dims, tensors)
        assert count == [(L - 1).bit_length() for L in dims]
        got = C.brute_force_sum(nb, [(vs, d) for vs, d in btens if vs] ) * np.prod(
            [complex(d) for vs, d in btens if not vs]) if nb else want
        assert abs(got - want) <= 1e-9 * max(abs(want), 1.0)
