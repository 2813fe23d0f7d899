"""Property tests of the CPU oracle on random small graphs and networks.

Invariants from the paper: the tree decomposition criteria (Sec. 2.2),
widths of orders vs the optimum, the removal bounds of Sec. 3.1 and the
slice-sum identity of Eq. 4; plus brute force as the plain definition of the
contraction.
"""
import numpy as np
from hypothesis import given, settings, strategies as st

from circuitgen import random_network
from oracle import contract as C
from oracle import planner as P


@st.composite
def graphs(draw, max_n=8):
    n = draw(st.integers(1, max_n))
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    chosen = draw(st.lists(st.sampled_from(pairs), unique=True, max_size=len(pairs))) if pairs else []
    adj = {v: set() for v in range(n)}
    for a, b in chosen:
        adj[a].add(b)
        adj[b].add(a)
    return adj


@settings(max_examples=150, deadline=None)
@given(graphs(), st.randoms(use_true_random=False))
def test_clique_tree_is_valid_td_of_width_of_order(adj, rnd):
    order = sorted(adj)
    rnd.shuffle(order)
    bags, parent = P.clique_tree(adj, order)
    assert P.is_valid_td(adj, bags, parent)
    assert P.td_width(bags) == P.treewidth_from_order(adj, order)
    # only maximal bags are kept (App. A)
    for i, b in enumerate(bags):
        assert not any(b < c for j, c in enumerate(bags) if j != i)


@settings(max_examples=120, deadline=None)
@given(graphs())
def test_min_fill_width_is_at_least_optimal(adj):
    order = P.min_fill_order(adj)
    assert sorted(order) == sorted(adj)
    assert P.treewidth_from_order(adj, order) >= P.optimal_treewidth(adj)


@settings(max_examples=120, deadline=None)
@given(graphs(max_n=7))
def test_optimal_treewidth_drops_at_most_one_and_is_monotone(adj):
    # Sec. 3.1: removing one vertex lowers the (optimal) treewidth by at most
    # one and never raises it.
    if len(adj) < 2:
        return
    tw = P.optimal_treewidth(adj)
    for u in list(adj):
        t2 = P.optimal_treewidth(P.remove_vertex(adj, u))
        assert tw - 1 <= t2 <= tw


@settings(max_examples=120, deadline=None)
@given(graphs(), st.randoms(use_true_random=False))
def test_reduced_order_never_widens(adj, rnd):
    # The filled graph of pi minus u on G minus u is a subgraph of the filled
    # graph of pi, so the width cannot grow.
    order = sorted(adj)
    rnd.shuffle(order)
    w = P.treewidth_from_order(adj, order)
    for u in order:
        red = [v for v in order if v != u]
        assert P.treewidth_from_order(P.remove_vertex(adj, u), red) <= w


@settings(max_examples=80, deadline=None)
@given(graphs(), st.integers(0, 4))
def test_alg2_returns_consistent_pieces(adj, m):
    order = P.min_fill_order(adj)
    m = min(m, len(adj))
    mu, g, pi, tau = P.greedy_treewidth_deletion(adj, order, m)
    assert len(mu) == m and len(set(mu)) == m
    assert pi == [v for v in order if v not in set(mu)]
    assert set(g) == set(adj) - set(mu)
    assert tau == P.treewidth_from_order(g, pi)
    assert tau <= P.treewidth_from_order(adj, order) if pi else True


@settings(max_examples=60, deadline=None)
@given(st.integers(2, 10), st.integers(1, 14), st.integers(1, 3), st.integers(0, 10**6), st.integers(0, 4))
def test_slicing_invariance_and_brute_force(n, t, r, seed, m):
    net = random_network(n, t, r, seed)
    tv = [v for v, _ in net.tensors]
    adj = P.simple_graph(n, tv)
    order = P.min_fill_order(adj)
    m = min(m, n)
    mu, _, pi, _ = P.greedy_treewidth_deletion(adj, order, m)
    want = C.brute_force_sum(n, net.tensors)
    unsliced, _ = C.contract(net.tensors, C.bucket_schedule(n, tv, order, []))
    sliced, vals = C.contract(net.tensors, C.bucket_schedule(n, tv, pi, mu))
    tol = 1e-11 * max(1.0, float(np.sum([np.abs(d).max() for _, d in net.tensors])) ** 2)
    assert abs(unsliced - want) <= tol * max(1.0, abs(want))
    assert abs(sliced - want) <= tol * max(1.0, abs(want))
    assert len(vals) == 1 << m


@settings(max_examples=40, deadline=None)
@given(st.integers(3, 9), st.integers(2, 12), st.integers(0, 10**6))
def test_any_order_gives_the_same_sum(n, t, seed):
    # The amplitude does not depend on the elimination order (Sec. 2.1).
    net = random_network(n, t, 3, seed)
    tv = [v for v, _ in net.tensors]
    rng = np.random.default_rng(seed)
    a, _ = C.contract(net.tensors, C.bucket_schedule(n, tv, list(range(n)), []))
    b, _ = C.contract(net.tensors, C.bucket_schedule(n, tv, [int(x) for x in rng.permutation(n)], []))
    assert abs(a - b) <= 1e-10 * max(1.0, abs(a))
