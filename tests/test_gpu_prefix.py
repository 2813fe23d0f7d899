"""Per-step plans with a fused prefix: the subtrees of small buckets run in one
LDS-resident launch of the fused executor, which writes the results larger
buckets read to the workspace; the per-step launches do the rest.  With
fused segments, later runs of small buckets also run as such launches,
reading the larger results they need from the workspace.  Neither changes
what the buckets compute, only where they run (Eqs. 2-4):
amplitudes and per-slice values must match the oracle at the parity
tolerance (relative 1e-5, per-slice values floored at 1e-5 of their RMS),
for whole and ragged slice ranges, small workspaces (several slice groups
per call), the reduced-precision MFMA forms and the allocation-free entry."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "amplitudes.json")
TOL = 1e-5


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as qbe
    return qbe, qbe.Context(0)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def check_slices(got, want):
    want = np.asarray(want)
    rms = float(np.sqrt(np.mean(np.abs(want) ** 2)))
    err = np.abs(np.asarray(got) - want)
    assert np.all(err <= TOL * np.maximum(np.abs(want), rms)), float(np.max(err / np.maximum(np.abs(want), rms)))


def golden_case(qbe, name, r, c, d):
    from circuitgen import circuit_model, random_grid_circuit
    g = json.load(open(GOLD))[name]
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(r, c, d, g["seed"])))
    return g, qm


def prefix_plan(qbe, ctx, qm, pi, mu, segments=False, **kw):
    plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step", fused_prefix=True, fused_segments=segments, **kw)
    st = plan.stats()
    assert st["prefix_buckets"] >= 2, st
    assert plan.launches()[0]["kind"] == "prefix"
    return plan


@pytest.mark.parametrize("segments", [False, True])
@pytest.mark.parametrize("name,shape,m", [("grid5x5_d16_m6", (5, 5, 16), 6), ("grid7x7_d24_m10", (7, 7, 24), 10)])
def test_prefix_plan_matches_oracle_slices_and_amplitude(env, name, shape, m, segments):
    qbe, ctx = env
    g, qm = golden_case(qbe, name, *shape)
    _, mu, pi, tau = qbe.plan_circuit(qm, m=m)
    assert tau == g["tau"]
    plan = prefix_plan(qbe, ctx, qm, pi, mu, segments)
    st = plan.stats()
    print(f"case prefix {name} segments={segments}: {st['fused_buckets']} buckets in "
          f"{st['n_fused_segments']} fused launches", flush=True)
    ws = plan.workspace()
    n = min(plan.n_slices, 64)
    _, per = qbe.qbe_contract_slices(ctx, plan, 0, n, ws)
    want = [complex(*v) for v in g["slices"]]
    check_slices(per[:len(want)], want[:n])
    assert rel(qbe.qbe_contract(ctx, plan, ws), complex(*g["oracle"])) <= TOL


@pytest.mark.parametrize("segments", [False, True])
@pytest.mark.parametrize("every", [1, 2])
def test_prefix_on_recomputed_plans(env, every, segments):
    """The headline's plan family: Alg. 2 with order recomputation on the
    7x7 depth-24 circuit (1024 slices), whose amplitude is fixed by the
    oracle whatever the schedule."""
    qbe, ctx = env
    g, qm = golden_case(qbe, "grid7x7_d24_m10", 7, 7, 24)
    mu, pi, _ = qbe.qbe_slice(qm, qbe.qbe_order_min_fill(qm), 10, recompute_every=every, tries=16, seed=2)
    plan = prefix_plan(qbe, ctx, qm, pi, mu, segments)
    if segments:
        assert plan.stats()["n_fused_segments"] >= 2
    print(f"case prefix 7x7 recompute every {every} segments={segments}", flush=True)
    ws = plan.workspace()
    got = qbe.qbe_contract(ctx, plan, ws)
    assert rel(got, complex(*g["oracle"])) <= TOL
    plain = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step")
    assert rel(got, qbe.qbe_contract(ctx, plain, plain.workspace())) <= TOL


@pytest.mark.parametrize("segments", [False, True])
def test_prefix_ragged_ranges_and_small_workspace(env, segments):
    """Slice groups that start anywhere: the fused launches read each
    slice's own inputs and the group's arena rows, and write its rows."""
    import torch
    qbe, ctx = env
    from circuitgen import circuit_model, random_grid_circuit
    from oracle import contract as C
    from oracle import planner as P
    mod = circuit_model(random_grid_circuit(4, 5, 12, 3))
    tv = [v for v, _ in mod.tensors]
    adj = P.simple_graph(mod.n_vars, tv)
    mu, _, pi, _ = P.greedy_treewidth_deletion(adj, P.min_fill_order(adj), 5)
    _, vals = C.contract(mod.tensors, C.bucket_schedule(mod.n_vars, tv, pi, mu))
    qm = qbe.Model.from_circuitgen(mod)
    plan = prefix_plan(qbe, ctx, qm, pi, mu, segments)
    st = plan.stats()
    ws = torch.empty(st["ws_bytes_min"] + 3 * (st["ws_bytes_all_slices"] - st["ws_bytes_min"]) // 32,
                     dtype=torch.uint8, device="cuda")
    for (b, e) in [(0, 32), (3, 17), (31, 32), (5, 6)]:
        print(f"case prefix ragged range {b}-{e} segments={segments}", flush=True)
        _, per = qbe.qbe_contract_slices(ctx, plan, b, e, ws)
        check_slices(per, vals[b:e])


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
def test_prefix_with_reduced_precision_mfma(env, prec):
    """The prefix computes in FP32 whatever the plan's precision; the
    per-step launches after it keep theirs.  Bounds as for the plain
    reduced-precision plans: bf16x6 at the FP32 tolerance, bf16x3 within
    7 chained products of 4 split terms at 2.5 * 2^-17 each."""
    qbe, ctx = env
    g, qm = golden_case(qbe, "grid5x5_d16_m6", 5, 5, 16)
    _, mu, pi, _ = qbe.plan_circuit(qm, m=6)
    plan = prefix_plan(qbe, ctx, qm, pi, mu, True, precision=prec)
    print(f"case prefix and segments {prec}", flush=True)
    got = qbe.qbe_contract(ctx, plan, plan.workspace())
    assert rel(got, complex(*g["oracle"])) <= (TOL if prec == "bf16x6" else 7 * 4 * 2.5 * 2.0 ** -17)


def test_prefix_static_entry_and_profile(env):
    """The allocation-free entry runs the same launches in the same order
    (same bits); per-launch timing lists the prefix first."""
    import torch
    qbe, ctx = env
    g, qm = golden_case(qbe, "grid7x7_d24_m10", 7, 7, 24)
    _, mu, pi, _ = qbe.plan_circuit(qm, m=10)
    plan = prefix_plan(qbe, ctx, qm, pi, mu, True)
    print("case prefix static entry", flush=True)
    ws = plan.workspace()
    want = qbe.qbe_contract(ctx, plan, ws)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    qbe.qbe_contract_static(ctx, plan, out)
    torch.cuda.synchronize()
    assert complex(*out.cpu().numpy()) == want
    ms = plan.profile(ws)
    assert len(ms) == len(plan.launches()) and np.all(ms >= 0.0)
    assert qbe.qbe_contract(ctx, plan, ws) == want


def test_prefix_plans_are_not_batched(env):
    qbe, ctx = env
    g, qm = golden_case(qbe, "grid5x5_d16_m6", 5, 5, 16)
    _, mu, pi, _ = qbe.plan_circuit(qm, m=6)
    plan = prefix_plan(qbe, ctx, qm, pi, mu, True)
    with pytest.raises(qbe.QbeError, match="INVALID_ARG"):
        qbe.Batch(ctx, [plan])
