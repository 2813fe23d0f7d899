"""Host planner behind the C ABI vs the CPU oracle: orders, widths, clique
trees, deletion sets and bucket schedules must agree exactly.  Runs on the
CPU (no device calls)."""
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import paper_2004_10892_amd as qbe
from circuitgen import (batch_instances, circuit_model, random_grid_circuit, random_network, toy_network)
from oracle import contract as C
from oracle import cost as K
from oracle import planner as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "qbe.h")).read()
    declared = set(re.findall(r"^\s*(?:int|int32_t|size_t|const char\*)\s+(qbe_\w+)\s*\(", header, re.M))
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(qbe._lib, name), name
    assert declared == set(qbe.EXPORTED)
    assert qbe.qbe_version() == 1


def test_close_is_safe_once_the_library_handle_is_cleared(monkeypatch):
    # at interpreter exit module globals may be cleared before finalisers
    # run; close() must then do nothing rather than raise
    m = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(3, 3, 4, 0)))
    assert m.handle
    monkeypatch.setattr(qbe, "_lib", None)
    m.close()
    assert m.handle  # nothing freed without the library
    monkeypatch.undo()
    m.close()
    assert m.handle is None


def oracle_plan(mod, m, score="tree_trimming"):
    tv = [v for v, _ in mod.tensors]
    adj = P.simple_graph(mod.n_vars, tv)
    order = P.min_fill_order(adj)
    mu, g, pi, tau = P.greedy_treewidth_deletion(adj, order, m, score=score)
    return adj, order, mu, pi, tau, C.bucket_schedule(mod.n_vars, tv, pi, mu)


CIRCUITS = [(3, 3, 6, s, 2) for s in range(8)] + [(4, 4, 10, s, 3) for s in range(8)] + \
           [(5, 5, 16, s, 6) for s in range(4)] + [(4, 6, 12, s, 4) for s in range(4)] + \
           [(6, 6, 16, 0, 8), (7, 7, 24, 0, 10)]


@pytest.mark.parametrize("rows,cols,depth,seed,m", CIRCUITS)
def test_plans_bit_exact_on_circuits(rows, cols, depth, seed, m):
    circ = random_grid_circuit(rows, cols, depth, seed)
    mod = circuit_model(circ)
    adj, order, mu, pi, tau, sched = oracle_plan(mod, m)
    qm = qbe.Model.from_circuitgen(mod)
    assert qbe.qbe_order_min_fill(qm) == order
    assert qbe.qbe_width(qm, order) == P.treewidth_from_order(adj, order)
    bags, parent = qbe.qbe_clique_tree(qm, order)
    obags, oparent = P.clique_tree(adj, order)
    assert bags == [sorted(b) for b in obags]
    assert parent == oparent
    qmu, qpi, qtau = qbe.qbe_slice(qm, order, m)
    assert (qmu, qpi, qtau) == (mu, pi, tau)
    assert qbe.qbe_width(qm, pi, removed=mu) == tau
    plan = qbe.Plan(qm, pi, mu)
    assert plan.dump() == C.schedule_dump(sched)
    stats = plan.stats()
    cost = K.schedule_cost(sched)
    assert stats["flops_per_slice"] == cost.flops_per_slice
    assert stats["bytes_per_slice"] == cost.bytes_per_slice
    assert stats["peak_bytes_per_slice"] == cost.peak_bytes
    assert stats["width"] == cost.width
    plan.check()


@pytest.mark.parametrize("score", ["degree", "tw_reduction", "betweenness"])
def test_other_scores_bit_exact(score):
    for seed in range(4):
        mod = circuit_model(random_grid_circuit(3, 4, 8, seed))
        _, order, mu, pi, tau, _ = oracle_plan(mod, 3, score=score)
        qm = qbe.Model.from_circuitgen(mod)
        assert qbe.qbe_slice(qm, order, 3, score=score) == (mu, pi, tau)


def test_target_width_mode():
    mod = circuit_model(random_grid_circuit(5, 5, 16, 1))
    tv = [v for v, _ in mod.tensors]
    adj = P.simple_graph(mod.n_vars, tv)
    order = P.min_fill_order(adj)
    mu, _, pi, tau = P.greedy_treewidth_deletion(adj, order, -1, target_width=6)
    qm = qbe.Model.from_circuitgen(mod)
    assert qbe.qbe_slice(qm, order, -1, target_width=6) == (mu, pi, tau)
    assert tau <= 6


@settings(max_examples=60, deadline=None)
@given(st.integers(2, 12), st.integers(1, 16), st.integers(1, 4), st.integers(0, 10**6), st.integers(0, 4))
def test_random_networks_bit_exact(n, t, r, seed, m):
    net = random_network(n, t, r, seed)
    m = min(m, n)
    adj, order, mu, pi, tau, sched = oracle_plan(net, m)
    qm = qbe.Model(net.n_vars, net.tensors)
    assert qbe.qbe_order_min_fill(qm) == order
    assert qbe.qbe_slice(qm, order, m) == (mu, pi, tau)
    plan = qbe.Plan(qm, pi, mu)
    assert plan.dump() == C.schedule_dump(sched)
    plan.check()


def test_toy_dump_through_abi_is_eq2():
    net = toy_network(0)
    qm = qbe.Model(net.n_vars, net.tensors)
    plan = qbe.Plan(qm, [0, 1, 2, 3, 4, 5], [])
    gold = "".join(l for l in open(os.path.join(ROOT, "tests", "golden", "toy_eq2_schedule.txt"))
                   if not l.startswith("#"))
    assert plan.dump() == gold
    assert qbe.qbe_slice(qm, [0, 1, 2, 3, 4, 5], 1) == ([2], [0, 1, 3, 4, 5], 1)


def test_fused_form_chosen_for_small_slices_and_per_step_for_large():
    mod = circuit_model(random_grid_circuit(5, 5, 16, 1))
    qm = qbe.Model.from_circuitgen(mod)
    _, mu, pi, _ = qbe.plan_circuit(qm, m=6)
    st_ = qbe.Plan(qm, pi, mu).stats()
    assert st_["exec"] == qbe.EXEC["fused"] and 0 < st_["lds_bytes"] <= 160 * 1024
    mod7 = circuit_model(random_grid_circuit(7, 7, 24, 0))
    q7 = qbe.Model.from_circuitgen(mod7)
    _, mu7, pi7, tau7 = qbe.plan_circuit(q7, m=10)
    st7 = qbe.Plan(q7, pi7, mu7).stats()
    assert st7["exec"] == qbe.EXEC["per_step"] and st7["width"] == tau7
    with pytest.raises(qbe.QbeError):
        qbe.Plan(q7, pi7, mu7, exec="fused")


@pytest.mark.parametrize("rows,cols,depth,seed,m", [(4, 4, 10, 0, 0), (5, 5, 16, 1, 6)])
def test_fused_program_merges_buckets_into_fewer_levels(rows, cols, depth, seed, m):
    # the fused program merges chains of buckets (several variables summed
    # per record); its level count drops below the buckets' dependency depth
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(rows, cols, depth, seed)))
    _, mu, pi, _ = qbe.plan_circuit(qm, m=m)
    plan = qbe.Plan(qm, pi, mu, exec="fused")
    plan.check()
    st_ = plan.stats()
    assert 0 < st_["fused_levels"] < st_["n_levels"]
    per_step = qbe.Plan(qm, pi, mu, exec="per_step").stats()
    assert per_step["fused_levels"] == st_["fused_levels"]  # the program exists either way


def test_batch_instance_plans_are_sound():
    """Every plan of the 512-instance batch workload passes the host check of
    every index its kernels can form, in both forms and without merging."""
    for (r, c, d, m, seed) in batch_instances(512):
        qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(r, c, d, seed)))
        _, mu, pi, _ = qbe.plan_circuit(qm, m=m)
        for kw in ({}, {"exec": "per_step"}, {"exec": "per_step", "merge": False}):
            plan = qbe.Plan(qm, pi, mu, **kw)
            plan.check()
            plan.close()


def test_invalid_arguments_return_errors():
    net = toy_network(0)
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        qbe.Model(3, [((0, 0), np.ones((2, 2)))])          # repeated variable
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        qbe.Model(4, [((0, 1), np.ones((2, 2)))])          # variables 2, 3 unused
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        qbe.Model(2, [((0, 5), np.ones((2, 2)))])          # id out of range
    qm = qbe.Model(net.n_vars, net.tensors)
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        qbe.qbe_width(qm, [0, 1, 2])                       # not a permutation
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        qbe.Plan(qm, [0, 1, 2, 3, 4], [])                  # variable 5 missing
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        qbe.Plan(qm, [0, 1, 2, 3, 4, 5], [2])              # sliced and ordered
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        qbe.qbe_slice(qm, [0, 1, 2, 3, 4, 5], 7)           # more than n


def test_no_device_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc = qbe._lib.qbe_create(qbe.C.byref(qbe._vp()), 0, None)
    assert rc == -6


def test_one_hip_runtime_in_process():
    # the package binds to the HIP runtime torch loaded; a second copy of the
    # runtime in the process would not see the device
    with open("/proc/self/maps") as f:
        maps = f.read()
    for name in ("libamdhip64", "libhsa-runtime64"):
        paths = {l.split()[-1] for l in maps.splitlines() if name in l}
        assert len(paths) == 1, paths


def test_host_clone_keeps_schedule_and_checks_structure():
    """A clone for another bitstring has the source plan's schedule and
    program statistics; a model of another structure is refused."""
    circ = random_grid_circuit(4, 4, 10, 5)
    a = qbe.Model.from_circuitgen(circuit_model(circ, 0))
    b = qbe.Model.from_circuitgen(circuit_model(circ, 0xFFFF))
    _, mu, pi, _ = qbe.plan_circuit(a, m=3)
    for form in ("fused", "per_step"):
        p = qbe.Plan(a, pi, mu, exec=form)
        c = p.clone(b)
        assert c.dump() == p.dump()
        assert c.stats() == p.stats()
        p.close()  # the clone does not depend on its source
        assert c.stats()["m"] == 3
        c.check()
    other = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(4, 4, 11, 5)))
    with pytest.raises(qbe.QbeError):
        qbe.Plan(a, pi, mu).clone(other)


def test_betweenness_bit_exact_on_larger_circuits():
    for (r, c, d, s, m) in [(5, 6, 16, 2, 6), (6, 6, 16, 3, 5)]:
        mod = circuit_model(random_grid_circuit(r, c, d, s))
        _, order, mu, pi, tau, _ = oracle_plan(mod, m, score="betweenness")
        qm = qbe.Model.from_circuitgen(mod)
        assert qbe.qbe_slice(qm, order, m, score="betweenness") == (mu, pi, tau)


def test_score_study_rows_follow_the_planner():
    """The study's rows are the planner's choices and the cost model's
    figures for every m; the greedy choices are prefix-consistent."""
    from paper_2004_10892_amd import study as S
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(4, 4, 10, 2)))
    res = S.study(qm, S.SCORES, m_max=4)
    order = qbe.qbe_order_min_fill(qm)
    widths0 = {rows[0]["width"] for rows in res.values()}
    assert len(widths0) == 1  # nothing removed: the same order for every score
    for score, rows in res.items():
        assert [r["m"] for r in rows] == list(range(5))
        for r in rows:
            mu, red, tau = qbe.qbe_slice(qm, order, r["m"], score=score)
            c = qbe.qbe_schedule_cost(qm, red, mu)
            assert r["mu"] == mu and r["width"] == tau
            assert r["flops_per_slice"] == c["flops_per_slice"]
            assert r["peak_bytes_per_slice"] == c["peak_bytes_per_slice"]
        assert rows[-1]["mu"][:3] == rows[3]["mu"]
    assert "| m |" in S.table(res)


def test_order_recomputation_bit_exact():
    """Alg. 5, the anytime order heuristic and Alg. 2 with recomputation
    through the C ABI against the oracle."""
    for (r, c, d, s, m, k) in [(4, 4, 10, 0, 4, 1), (4, 5, 12, 1, 5, 2), (5, 5, 12, 2, 6, 3)]:
        mod = circuit_model(random_grid_circuit(r, c, d, s))
        adj = P.simple_graph(mod.n_vars, [v for v, _ in mod.tensors])
        order = P.min_fill_order(adj)
        qm = qbe.Model.from_circuitgen(mod)
        bags, parent = P.clique_tree(adj, order)
        assert qbe.qbe_order_from_td(mod.n_vars, [sorted(b) for b in bags], parent) == P.recover_order(bags, parent)
        want = P.anytime_order(adj, 5, 99)
        assert qbe.qbe_order_anytime(qm, (), 5, 99) == (want, P.treewidth_from_order(adj, want))
        mu, _, pi, tau = P.greedy_treewidth_deletion_recompute(adj, order, m, k, 3, 7)
        assert qbe.qbe_slice(qm, order, m, recompute_every=k, tries=3, seed=7) == (mu, pi, tau)


def test_order_from_td_rejects_bad_decompositions():
    with pytest.raises(qbe.QbeError):
        qbe.qbe_order_from_td(3, [[0, 1], [1, 2]], [1, 0])  # cycle
    with pytest.raises(qbe.QbeError):
        qbe.qbe_order_from_td(3, [[0, 1], [1, 2], [0, 2]], [1, -1, 1])  # 0 in two subtrees
    with pytest.raises(qbe.QbeError):
        qbe.qbe_order_from_td(3, [[0, 5]], [-1])  # id out of range
    assert qbe.qbe_order_from_td(3, [[0, 1], [1, 2]], [1, -1]) == [0, 1, 2]


def test_general_dimension_models_expand_to_binary():
    """qbe_model_create_dims: variable v of dimension L becomes ceil(log2 L)
    consecutive binary variables; the expanded model has the oracle's
    expansion's structure (its min-fill order and clique tree are the
    oracle's on that expansion) and its plans pass the host check."""
    from circuitgen import random_general_network
    from oracle import general as Gn
    for seed in range(6):
        dims, tensors = random_general_network(seed)
        qm = qbe.Model.from_dims(dims, tensors)
        nb, btens, first, count = Gn.binary_expansion(dims, tensors)
        assert qm.n_vars == nb
        assert [qm.var_bits(v) for v in range(len(dims))] == list(zip(first, count))
        adj = P.simple_graph(nb, [vs for vs, _ in btens])
        order = qbe.qbe_order_min_fill(qm)
        assert order == P.min_fill_order(adj)
        m = min(2, nb)
        mu, pi, tau = qbe.qbe_slice(qm, order, m)
        for form in ("per_step", "auto"):
            plan = qbe.Plan(qm, pi, mu, exec=form)
            plan.check()
            plan.close()
    with pytest.raises(qbe.QbeError):
        qbe.Model.from_dims([3, 0], [((0, 1), np.ones((3, 0)))])  # dimension 0
    with pytest.raises(qbe.QbeError):
        qbe.Model.from_dims([2 ** 16, 2 ** 16, 2 ** 16], [((0, 1, 2), np.ones(1))])  # 48 bits
    b = qbe.Model(3, [((0, 1), np.ones((2, 2))), ((2,), np.ones(2))])
    assert b.var_bits(2) == (2, 1)


def test_fused_programs_of_degenerate_schedules():
    """Schedules with no buckets (every variable sliced) or a single one
    still compile to sound fused programs (only scalar factors, or one
    level), as the per-step form does."""
    rng = np.random.default_rng(3)
    t = [((0, 1), rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))),
         ((1,), rng.standard_normal(2) + 0j)]
    qm = qbe.Model(2, t)
    for mu, order in (([0, 1], []), ([1], [0]), ([], [0, 1])):
        for form in ("fused", "per_step"):
            plan = qbe.Plan(qm, order, mu, exec=form)
            plan.check()
            assert plan.stats()["exec"] == qbe.EXEC[form]
        if not order:
            assert qbe.Plan(qm, order, mu, exec="fused").stats()["fused_levels"] == 0
