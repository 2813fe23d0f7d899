"""Planner reference: graphs, elimination orders, tree decompositions and the
greedy mu-treewidth deletion -- TEST INFRASTRUCTURE (see package header).

Readings of points the paper leaves open:

* Graphs are simple (Sec. 2.2, footnote): a tensor is a clique over its
  variables; self-loops are dropped and parallel edges merged.
* Greedy min-fill order: repeatedly eliminate the vertex whose elimination
  adds the fewest edges in the current elimination graph; ties go to the
  smaller current degree, then to the smaller vertex id.
* Alg. 1 (Sec. 2.3) returns tau = max |N(u)| over the elimination, where
  N(u) are the not-yet-eliminated neighbours of u in the filled graph.  The
  listing starts from tau = 1 and has no return; the plain maximum is
  returned here (0 for an edgeless graph).
* Alg. 4 (App. A) is read through the text under it: the tree consists of
  the *maximal* cliques {u} + N+(u) of the elimination.  A bag {u} + N+(u)
  is maximal unless an elimination-tree child w of u has |N+(w)| equal to
  its size (Blair and Peyton's criterion, the reference the appendix cites).
  An isolated vertex gets the bag {u}.
* Tree-trimming (Sec. 3.2): b_max is the union of all bags of maximum size;
  the "length" of the subtree S_u is the number of bags holding u, its
  weight the sum of their sizes; the largest (length, weight) wins and a
  remaining tie goes to the vertex eliminated earliest in the current order
  (instead of a random pick).  After each removal the tree is rebuilt from
  the reduced graph and the reduced order.
* Alg. 2 (Sec. 3): the score is per vertex; the optional recomputation of
  the order that Alg. 2 allows after each removal is not performed, so the reduced order is the
  original order with mu removed.  It stops after m removals or, when m is
  negative, as soon as the width of the reduced order is at most a target.
* Alg. 3 (Sec. 3.1): the reduced graph is G minus u (the listing writes
  u*), the best drop found so far is updated, vertices are scanned in order
  of the elimination order, and when no removal reduces the width the first
  vertex of the order is returned.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Sequence, Tuple

Adj = Dict[int, set]


# ------------------------------------------------------------------ graphs --

def simple_graph(n_vars: int, tensor_vars: Iterable[Sequence[int]]) -> Adj:
    """Simple undirected graph of a network: every tensor is a clique."""
    adj: Adj = {v: set() for v in range(n_vars)}
    for vs in tensor_vars:
        for a in vs:
            for b in vs:
                if a != b:
                    adj[a].add(b)
    return adj


def copy_graph(adj: Adj) -> Adj:
    return {v: set(ns) for v, ns in adj.items()}


def remove_vertex(adj: Adj, u: int) -> Adj:
    """G minus u (Sec. 2.4: fixing an index removes its vertex)."""
    g = {v: set(ns) for v, ns in adj.items() if v != u}
    for ns in g.values():
        ns.discard(u)
    return g


# ------------------------------------------------------ elimination basics --

def eliminate(adj: Adj, order: Sequence[int]) -> List[Tuple[int, frozenset]]:
    """Eliminate vertices along ``order``; return (u, N+(u)) per step.

    N+(u) is the set of not-yet-eliminated neighbours of u at the moment u is
    eliminated; those neighbours are then joined into a clique (Sec. 2.1, the
    step described under Eq. 2).
    """
    if sorted(order) != sorted(adj):
        raise ValueError("order must be a permutation of the graph's vertices")
    g = copy_graph(adj)
    out = []
    for u in order:
        nbrs = frozenset(g[u])
        for w in nbrs:
            g[w] |= nbrs
            g[w].discard(w)
            g[w].discard(u)
        del g[u]
        out.append((u, nbrs))
    return out


def treewidth_from_order(adj: Adj, order: Sequence[int]) -> int:
    """Alg. 1: the largest neighbourhood met while eliminating along ``order``."""
    tau = 0
    for _, nbrs in eliminate(adj, order):
        tau = max(tau, len(nbrs))
    return tau


def min_fill_order(adj: Adj) -> List[int]:
    """Greedy min-fill elimination order (ties: smaller degree, smaller id).

    Adjacency is kept as integer bit masks.  After eliminating u only the
    vertices within distance two of u can change their fill value (their
    neighbourhood changed, or two of their neighbours were joined), so only
    those are re-scored.
    """
    verts = sorted(adj)
    nb = {v: 0 for v in verts}
    for v in verts:
        for w in adj[v]:
            nb[v] |= 1 << w

    def members(mask: int):
        while mask:
            low = mask & -mask
            yield low.bit_length() - 1
            mask ^= low

    def fill(v: int) -> int:
        d = nb[v].bit_count()
        inner = sum((nb[w] & nb[v]).bit_count() for w in members(nb[v]))
        return d * (d - 1) // 2 - inner // 2

    score = {v: fill(v) for v in verts}
    alive = set(verts)
    order = []
    while alive:
        u = min(alive, key=lambda v: (score[v], nb[v].bit_count(), v))
        order.append(u)
        nu = nb[u]
        bit_u = 1 << u
        for w in members(nu):
            nb[w] = (nb[w] | nu) & ~(1 << w) & ~bit_u
        nb[u] = 0
        alive.discard(u)
        del score[u]
        touched = set(members(nu))
        for w in list(touched):
            touched.update(members(nb[w]))
        for v in touched:
            score[v] = fill(v)
    return order


# ------------------------------------------------------- clique tree (A) --

def clique_tree(adj: Adj, order: Sequence[int]):
    """Tree decomposition of App. A from an elimination order.

    Returns ``(bags, parent)``: ``bags`` lists the maximal cliques as
    frozensets, ordered by the position of their earliest-eliminated vertex;
    ``parent[i]`` is the index of the parent bag (``-1`` for a root).  A
    disconnected graph yields a forest (one root per component).
    """
    elim = eliminate(adj, order)
    pos = {u: i for i, u in enumerate(order)}
    nplus = {u: n for u, n in elim}
    bag = {u: frozenset({u}) | nplus[u] for u in order}
    etree_parent = {}
    children = {u: [] for u in order}
    for u in order:
        if nplus[u]:
            p = min(nplus[u], key=pos.__getitem__)
            etree_parent[u] = p
            children[p].append(u)
    maximal = {}
    rep = {}
    for u in order:  # children precede their parent in the order
        absorbed_by = [w for w in children[u] if len(nplus[w]) == len(bag[u])]
        maximal[u] = not absorbed_by
        rep[u] = u if maximal[u] else rep[absorbed_by[0]]
    reps = [u for u in order if maximal[u]]
    index = {u: i for i, u in enumerate(reps)}
    bags = [bag[u] for u in reps]
    # The vertices absorbed into the bag of u form a chain above u in the
    # elimination tree; the bag's parent is the bag of the vertex above the
    # top of that chain.
    parent = []
    for u in reps:
        x = u
        while x in etree_parent and rep[etree_parent[x]] == u:
            x = etree_parent[x]
        parent.append(index[rep[etree_parent[x]]] if x in etree_parent else -1)
    return bags, parent


def td_width(bags) -> int:
    """Width of a tree decomposition: largest bag size minus one (Sec. 2.3)."""
    return max(len(b) for b in bags) - 1 if bags else -1


def is_valid_td(adj: Adj, bags, parent) -> bool:
    """The three criteria of Sec. 2.2 plus the tree (forest) shape."""
    verts = set(adj)
    covered = set().union(*bags) if bags else set()
    if covered != verts:
        return False
    for u in adj:
        for w in adj[u]:
            if not any(u in b and w in b for b in bags):
                return False
    # parent array must describe a forest
    for i in range(len(bags)):
        seen = set()
        j = i
        while j != -1:
            if j in seen:
                return False
            seen.add(j)
            j = parent[j]
    # running intersection: bags holding u form one connected subtree
    for u in verts:
        holding = [i for i, b in enumerate(bags) if u in b]
        tops = [i for i in holding if parent[i] == -1 or u not in bags[parent[i]]]
        if len(tops) != 1:
            return False
    return True


# ------------------------------------------------------------------ scores --

def tree_trimming_pick(adj: Adj, order: Sequence[int]) -> int:
    """Sec. 3.2: the vertex of the maximum bags with the longest, then
    heaviest, subtree; remaining ties go to the earliest vertex in ``order``."""
    bags, _ = clique_tree(adj, order)
    smax = max(len(b) for b in bags)
    bmax = set().union(*[b for b in bags if len(b) == smax])
    pos = {u: i for i, u in enumerate(order)}
    best = None
    for u in bmax:
        length = sum(1 for b in bags if u in b)
        weight = sum(len(b) for b in bags if u in b)
        key = (length, weight, -pos[u])
        if best is None or key > best[0]:
            best = (key, u)
    return best[1]


def degree_pick(adj: Adj, order: Sequence[int]) -> int:
    """Sec. 3.1 degree score; ties go to the earliest vertex in ``order``."""
    pos = {u: i for i, u in enumerate(order)}
    return max(adj, key=lambda u: (len(adj[u]), -pos[u]))


def betweenness_pick(adj: Adj, order: Sequence[int]) -> int:
    """Sec. 3.1 betweenness-centrality score (networkx, unnormalised)."""
    import networkx as nx

    g = nx.Graph()
    g.add_nodes_from(adj)
    for u, ns in adj.items():
        for w in ns:
            if u < w:
                g.add_edge(u, w)
    bc = nx.betweenness_centrality(g, normalized=False)
    pos = {u: i for i, u in enumerate(order)}
    return max(adj, key=lambda u: (round(bc[u], 9), -pos[u]))


def tw_reduction_pick(adj: Adj, order: Sequence[int]) -> int:
    """Alg. 3: the vertex whose removal lowers the order's width the most."""
    tau = treewidth_from_order(adj, order)
    delta = 0
    best = order[0]
    for u in order:
        reduced = [v for v in order if v != u]
        d = tau - treewidth_from_order(remove_vertex(adj, u), reduced)
        if d > delta:
            delta = d
            best = u
    return best


SCORES = {
    "tree_trimming": tree_trimming_pick,
    "degree": degree_pick,
    "betweenness": betweenness_pick,
    "tw_reduction": tw_reduction_pick,
}


def greedy_treewidth_deletion(adj: Adj, order: Sequence[int], m: int,
                              target_width: int = -1, score: str = "tree_trimming"):
    """Alg. 2.  Returns ``(mu, reduced_graph, reduced_order, tau)``.

    ``mu`` lists the removed vertices in the order they were chosen.  With
    ``m >= 0`` exactly ``m`` vertices are removed; with ``m < 0`` vertices are
    removed until the width of the reduced order is at most ``target_width``.
    """
    pick = SCORES[score]
    g = copy_graph(adj)
    pi = list(order)
    mu: List[int] = []
    while pi:
        if m >= 0 and len(mu) >= m:
            break
        if m < 0 and treewidth_from_order(g, pi) <= target_width:
            break
        u = pick(g, pi)
        g = remove_vertex(g, u)
        pi.remove(u)
        mu.append(u)
    if m >= 0 and len(mu) < m:
        raise ValueError("cannot remove more vertices than the graph has")
    return mu, g, pi, treewidth_from_order(g, pi)


# ------------------------------------------ order recomputation (Alg. 2, 5) --

def recover_order(bags, parent) -> List[int]:
    """App. B, Alg. 5: an elimination order consistent with a tree
    decomposition.  Repeatedly the first bag (in index order) that is a leaf
    and not a root is taken; the vertices it has and its parent lacks go to
    the order (ascending ids; the algorithm allows any order), and the leaf
    is removed.  The roots' vertices come last (a forest: root by root)."""
    nb = len(bags)
    alive = [True] * nb
    children = [0] * nb
    for i, p in enumerate(parent):
        if p >= 0:
            children[p] += 1
    order: List[int] = []
    while True:
        leaf = next((i for i in range(nb) if alive[i] and parent[i] >= 0 and children[i] == 0), None)
        if leaf is None:
            break
        order += sorted(set(bags[leaf]) - set(bags[parent[leaf]]))
        alive[leaf] = False
        children[parent[leaf]] -= 1
    for i in range(nb):
        if alive[i]:
            order += sorted(bags[i])
    return order


class _SplitMix64:
    """SplitMix64 (Steele, Lea and Flood, 2014)."""

    def __init__(self, seed: int):
        self.state = seed & 0xFFFFFFFFFFFFFFFF

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
        return z ^ (z >> 31)


def _min_fill_with(adj: Adj, prio: Dict[int, int]) -> List[int]:
    """Greedy min-fill; ties in (fill, degree) go to the smaller prio[v]."""
    verts = sorted(adj)
    nb = {v: set(adj[v]) for v in verts}
    alive = set(verts)
    order = []

    def fill(v):
        ns = nb[v]
        d = len(ns)
        inner = sum(len(nb[w] & ns) for w in ns)
        return d * (d - 1) // 2 - inner // 2

    while alive:
        u = min(alive, key=lambda v: (fill(v), len(nb[v]), prio[v]))
        order.append(u)
        for w in nb[u]:
            nb[w] |= nb[u]
            nb[w].discard(w)
            nb[w].discard(u)
        nb[u] = set()
        alive.discard(u)
    return order


def anytime_order(adj: Adj, tries: int, seed: int) -> List[int]:
    """The project's anytime tree-decomposition heuristic (it stands in for
    the external solver of Sec. 4): try 0 is greedy min-fill (ties: degree,
    id); try t >= 1 breaks (fill, degree) ties by random priorities drawn
    from one SplitMix64(seed) stream, one draw per vertex in ascending id
    order per try.  The first order of smallest width wins."""
    rng = _SplitMix64(seed)
    best = min_fill_order(adj)
    bw = treewidth_from_order(adj, best)
    for _ in range(1, tries):
        prio = {v: rng.next() for v in sorted(adj)}
        o = _min_fill_with(adj, prio)
        w = treewidth_from_order(adj, o)
        if w < bw:
            best, bw = o, w
    return best


def greedy_treewidth_deletion_recompute(adj: Adj, order: Sequence[int], m: int, recompute_every: int,
                                        tries: int, seed: int, target_width: int = -1,
                                        score: str = "tree_trimming"):
    """Alg. 2 with its optional line: after every ``recompute_every``-th
    removal the reduced order is recomputed -- the anytime heuristic's
    order on the reduced graph, turned into its tree decomposition (App. A)
    and back into an order by Alg. 5.  Returns ``(mu, reduced_graph,
    reduced_order, tau)``."""
    pick = SCORES[score]
    g = copy_graph(adj)
    pi = list(order)
    mu: List[int] = []
    while pi:
        if m >= 0 and len(mu) >= m:
            break
        if m < 0 and treewidth_from_order(g, pi) <= target_width:
            break
        u = pick(g, pi)
        g = remove_vertex(g, u)
        pi.remove(u)
        mu.append(u)
        if recompute_every > 0 and len(mu) % recompute_every == 0 and pi:
            bags, parent = clique_tree(g, anytime_order(g, tries, seed))
            pi = recover_order(bags, parent)
    if m >= 0 and len(mu) < m:
        raise ValueError("cannot remove more vertices than the graph has")
    return mu, g, pi, treewidth_from_order(g, pi)


def optimal_treewidth(adj: Adj) -> int:
    """Brute-force treewidth: minimum width over all elimination orders.

    Only for tiny graphs (<= 8 vertices).  Uses the fact that the best order
    can be found by dynamic programming over eliminated subsets: the width of
    eliminating u after the set S is the number of vertices outside S + {u}
    reachable from u through S (Bodlaender et al.'s formulation).
    """
    verts = sorted(adj)
    n = len(verts)
    if n == 0:
        return -1
    if n > 12:
        raise ValueError("brute force only for tiny graphs")
    idx = {v: i for i, v in enumerate(verts)}

    def q_value(s_mask: int, u: int) -> int:
        # vertices not in S + {u} reachable from u via paths inside S
        seen = {u}
        stack = [u]
        out = set()
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if y in seen:
                    continue
                seen.add(y)
                if s_mask >> idx[y] & 1:
                    stack.append(y)
                else:
                    out.add(y)
        return len(out)

    full = (1 << n) - 1
    best = {0: -1}
    for s in range(1 << n):
        if s not in best:
            continue
        for u in verts:
            bit = 1 << idx[u]
            if s & bit:
                continue
            w = max(best[s], q_value(s, u))
            t = s | bit
            if t not in best or w < best[t]:
                best[t] = w
    return max(best[full], 0)
