"""Hand-worked pins of the oracle's remaining planner parts: the degree
score (Sec. 3.1), the direct width-reduction score (Alg. 3), Alg. 2's
optional order recomputation with Alg. 5 (App. B), the tree-decomposition
criteria (Sec. 2.2) and the incremental rescoring of greedy min-fill.

Every expected value below is derived by hand in the comment above it; each
case is chosen so that a plausible wrong variant (a Delta that is never
updated, >= instead of >, ties to the smallest id, no recomputation, an
always-true validity check, stale fill values) gives another answer."""
import pytest

from oracle import planner as P


def graph(n_vertices, edges):
    adj = {v: set() for v in range(n_vertices)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    return adj


# Star s = 0 with leaves 1..5, and a K4 on a, b, c, d = 6, 7, 8, 9.
STAR_K4 = graph(10, [(0, i) for i in range(1, 6)] + [(6, 7), (6, 8), (6, 9), (7, 8), (7, 9), (8, 9)])
STAR_K4_ORDER = [1, 2, 3, 4, 5, 0, 6, 7, 8, 9]


def test_width_of_star_k4_order():
    # leaves: N+ = {s} (1); s: none left (0); a: {b, c, d} (3); b: 2; c: 1
    assert P.treewidth_from_order(STAR_K4, STAR_K4_ORDER) == 3


def test_degree_and_alg3_pick_different_vertices():
    # degree: s has 5 neighbours, a..d have 3 -> s
    assert P.degree_pick(STAR_K4, STAR_K4_ORDER) == 0
    # Alg. 3: removing s leaves the K4 (width 3, drop 0); removing a vertex
    # of the K4 leaves a triangle (width 2, drop 1); leaves drop 0.  Scanned
    # in the order, a (= 6) is the first with drop 1 > 0 and b, c, d only tie
    # it, so a.  (A Delta that is never updated, or >= in place of >, ends
    # on d = 9.)
    assert P.tw_reduction_pick(STAR_K4, STAR_K4_ORDER) == 6


# Hub h = 0 with neighbours x1..x4 = 1..4 (independent), and a triangle
# a, b, c = 5, 6, 7.  Order: h first, then the x's, then the triangle.
HUB = graph(8, [(0, 1), (0, 2), (0, 3), (0, 4), (5, 6), (5, 7), (6, 7)])
HUB_ORDER = [0, 1, 2, 3, 4, 5, 6, 7]


def test_alg3_updates_delta():
    # width: h has N+ = {x1..x4} (4), which become a clique; x1: 3, x2: 2 ..;
    # a: 2 -> width 4.  Remove h: the x's stay independent (0), the triangle
    # gives 2 -> drop 2.  Remove x_i: h has 3 left -> width 3, drop 1.
    # Remove a triangle vertex: still 4, drop 0.  Scan: h (2), then x1..x4
    # (1 each, not above 2) -> h.  Without the update of Delta every x_i
    # has drop 1 > 0 and the last one, x4 = 4, would win.
    assert P.treewidth_from_order(HUB, HUB_ORDER) == 4
    assert P.tw_reduction_pick(HUB, HUB_ORDER) == 0


def test_alg3_without_improvement_returns_first_in_order():
    # two disjoint triangles: removing any vertex leaves the other triangle
    # (width 2 before and after) -> no drop -> the order's first vertex
    adj = graph(6, [(0, 1), (0, 2), (1, 2), (3, 4), (3, 5), (4, 5)])
    order = [4, 0, 1, 2, 3, 5]
    assert P.tw_reduction_pick(adj, order) == 4


def test_degree_ties_go_to_earliest_in_order():
    # two stars: s1 = 0 (leaves 1, 2, 3), s2 = 4 (leaves 5, 6, 7); equal
    # degree 3; s2 comes first in the order -> s2 (ties to the smallest id
    # would give 0)
    adj = graph(8, [(0, 1), (0, 2), (0, 3), (4, 5), (4, 6), (4, 7)])
    order = [5, 6, 7, 4, 1, 2, 3, 0]
    assert P.degree_pick(adj, order) == 4


def test_alg2_with_degree_and_alg3_scores():
    # degree: s first; in G minus s the K4 vertices have degree 3, the
    # leaves 0 -> a, the first of the K4 in the order
    mu, _, pi, tau = P.greedy_treewidth_deletion(STAR_K4, STAR_K4_ORDER, 2, score="degree")
    assert mu == [0, 6]
    assert pi == [1, 2, 3, 4, 5, 7, 8, 9]
    assert tau == 2  # a triangle b, c, d remains
    # Alg. 3: a first (above); then the triangle b, c, d: each removal drops
    # the width 2 -> 1, b first in the order
    mu, _, pi, tau = P.greedy_treewidth_deletion(STAR_K4, STAR_K4_ORDER, 2, score="tw_reduction")
    assert mu == [6, 7]
    assert tau == 1


def test_recomputation_changes_the_reduced_order():
    # Path 0-1-2-3-4, order [4, 3, 1, 0, 2], degree score, recompute after
    # every removal with one try (the anytime heuristic is plain min-fill).
    # Degree: 1, 2, 3 have degree 2; 3 comes first in the order -> mu = [3].
    # G minus 3 = path 0-1-2 plus the isolated 4; pi minus mu = [4, 1, 0, 2]
    # has width 2 (1 is eliminated with neighbours 0 and 2).
    # Min-fill on G minus 3: fills 0, 1, 0 for 0, 1, 2 and 0 for 4; among the
    # fill-0 vertices 4 has the smallest degree -> 4; then 0 (fill 0, degree
    # 1, smaller id than 2); then 1 (now fill 0, degree 1); then 2:
    # [4, 0, 1, 2].  Its clique tree (App. A): bags {4}, {0,1}, {1,2} ({2}
    # is absorbed by {1,2}); parents -1, 2, -1.  Alg. 5: the only non-root
    # leaf is {0,1}: it gives 0 (its parent {1,2} lacks it); the roots
    # follow, {4} then {1,2}: reduced order [0, 4, 1, 2], width 1.
    adj = graph(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    order = [4, 3, 1, 0, 2]
    mu, g, pi, tau = P.greedy_treewidth_deletion(adj, order, 1, score="degree")
    assert (mu, pi, tau) == ([3], [4, 1, 0, 2], 2)
    mu, g, pi, tau = P.greedy_treewidth_deletion_recompute(adj, order, 1, recompute_every=1, tries=1, seed=0,
                                                           score="degree")
    assert mu == [3]
    assert P.min_fill_order(g) == [4, 0, 1, 2]
    bags, parent = P.clique_tree(g, [4, 0, 1, 2])
    assert [sorted(b) for b in bags] == [[4], [0, 1], [1, 2]] and parent == [-1, 2, -1]
    assert pi == [0, 4, 1, 2]
    assert tau == 1


def test_is_valid_td_rejects_broken_decompositions():
    # path 0-1-2-3: a valid decomposition is {0,1} - {1,2} - {2,3}
    adj = graph(4, [(0, 1), (1, 2), (2, 3)])
    good = [frozenset({0, 1}), frozenset({1, 2}), frozenset({2, 3})]
    assert P.is_valid_td(adj, good, [1, 2, -1])
    # a vertex in no bag
    assert not P.is_valid_td(adj, [frozenset({0, 1}), frozenset({1, 2})], [1, -1])
    # the edge 2-3 in no bag (3 is covered by a bag of its own)
    assert not P.is_valid_td(adj, [frozenset({0, 1}), frozenset({1, 2}), frozenset({3})], [1, 2, -1])
    # running intersection broken: 1 in the first and last bag but not the middle
    bad_ri = [frozenset({0, 1}), frozenset({0, 2, 3}), frozenset({1, 2})]
    assert not P.is_valid_td(adj, bad_ri, [1, 2, -1])
    # parent array with a cycle
    assert not P.is_valid_td(adj, good, [1, 0, -1])
    # two roots holding the same vertex (a forest whose trees share vertex 1)
    assert not P.is_valid_td(adj, [frozenset({0, 1}), frozenset({1, 2, 3})], [-1, -1])


@pytest.mark.parametrize("rows,cols,depth,seed", [(3, 3, 8, 0), (4, 4, 10, 0), (5, 5, 16, 1)])
def test_incremental_min_fill_equals_plain_rescoring(rows, cols, depth, seed):
    """min_fill_order re-scores only the vertices near the eliminated one;
    _min_fill_with re-scores every vertex at every step.  With priority =
    id both apply the same rule (fill, degree, id), so the orders agree."""
    from circuitgen import circuit_model, random_grid_circuit
    mod = circuit_model(random_grid_circuit(rows, cols, depth, seed))
    adj = P.simple_graph(mod.n_vars, [v for v, _ in mod.tensors])
    assert P.min_fill_order(adj) == P._min_fill_with(adj, {v: v for v in adj})
