"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerance: the amplitude of a slice sum must match the complex128 oracle to
a relative error of 1e-5 (the accuracy target for complex64 arithmetic with
an FP64 slice sum).  Per-slice values are compared with the same relative
bound, floored at 1e-5 of the root-mean-square slice value (a slice that is
tiny because of cancellation carries the absolute error of its larger
neighbours).  Plans (orders, mu, schedules) are compared exactly.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-5


@pytest.fixture(scope="module")
def qbe():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as q
    return q


@pytest.fixture(scope="module")
def ctx(qbe):
    return qbe.Context(0)


def _say(*a):
    print(*a, flush=True)


def oracle_schedule(mod, m):
    from oracle import contract as C
    from oracle import planner as P
    tv = [v for v, _ in mod.tensors]
    adj = P.simple_graph(mod.n_vars, tv)
    order = P.min_fill_order(adj)
    mu, _, pi, _ = P.greedy_treewidth_deletion(adj, order, m)
    return mu, pi, C.bucket_schedule(mod.n_vars, tv, pi, mu)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def check_slices(got, want):
    want = np.asarray(want)
    rms = float(np.sqrt(np.mean(np.abs(want) ** 2)))
    err = np.abs(np.asarray(got) - want)
    bound = TOL * np.maximum(np.abs(want), rms)
    assert np.all(err <= bound), (float(np.max(err / np.maximum(np.abs(want), rms))))


WORK = {"grid4x4_d10_m0": (4, 4, 10, 0), "grid5x5_d16_m6": (5, 5, 16, 6)}


@pytest.mark.parametrize("form", ["fused", "per_step"])
@pytest.mark.parametrize("name", list(WORK))
def test_golden_workloads(qbe, ctx, name, form):
    from circuitgen import circuit_model, random_grid_circuit
    gold = json.load(open(os.path.join(GOLD, "amplitudes.json")))[name]
    r, c, d, m = WORK[name]
    mod = circuit_model(random_grid_circuit(r, c, d, gold["seed"]))
    qm = qbe.Model.from_circuitgen(mod)
    _, mu, pi, tau = qbe.plan_circuit(qm, m=m)
    assert tau == gold["tau"]
    _say(f"case {name} {form} m={m} tau={tau}")
    plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec=form)
    ws = plan.workspace()
    total, per = qbe.qbe_contract_slices(ctx, plan, 0, plan.n_slices, ws)
    want_sv = complex(*gold["statevector"])
    want_or = complex(*gold["oracle"])
    assert rel(total, want_or) <= TOL
    assert rel(total, want_sv) <= TOL
    check_slices(per, [complex(*v) for v in gold["slices"]])
    assert rel(qbe.qbe_contract(ctx, plan, ws), want_or) <= TOL


def test_7x7_d24_sampled_slices_and_full_amplitude(qbe, ctx):
    """Full size of the precision workload: slices 0..15 one by one against
    the oracle's stored values, and the sum of all 1024 slices."""
    import torch
    from circuitgen import circuit_model, random_grid_circuit
    gold = json.load(open(os.path.join(GOLD, "amplitudes.json")))["grid7x7_d24_m10"]
    mod = circuit_model(random_grid_circuit(7, 7, 24, gold["seed"]))
    qm = qbe.Model.from_circuitgen(mod)
    _, mu, pi, tau = qbe.plan_circuit(qm, m=10)
    assert tau == gold["tau"]
    _say(f"case 7x7 d24 m=10 tau={tau}")
    plan = qbe.Plan(qm, pi, mu, ctx=ctx)
    st = plan.stats()
    assert st["exec"] == qbe.EXEC["per_step"]
    ws = plan.workspace(all_slices=False)
    _, per = qbe.qbe_contract_slices(ctx, plan, 0, 16, ws)
    want = [complex(*v) for v in gold["slices"]]
    check_slices(per, want[:16])
    ws_all = torch.empty(min(st["ws_bytes_all_slices"], 64 << 30), dtype=torch.uint8, device="cuda")
    total = qbe.qbe_contract(ctx, plan, ws_all)
    assert rel(total, complex(*gold["oracle"])) <= TOL
    _say("case 7x7 autotuned")
    n_mfma = st["n_mfma_steps"]
    plan.autotune(ws_all)
    tuned = qbe.qbe_contract(ctx, plan, ws_all)
    assert rel(tuned, complex(*gold["oracle"])) <= TOL
    if plan.stats()["n_mfma_steps"] == n_mfma:
        # tile shapes changed, the arithmetic per entry did not
        assert tuned == total
    else:
        # merged launches moved between the MFMA and the VALU kernels (both
        # FP32 products, other rounding order of the sums)
        _say(f"  {n_mfma - plan.stats()['n_mfma_steps']} merged launches moved to the VALU kernels")


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("form", ["fused", "per_step"])
def test_random_networks_vs_brute_force(qbe, ctx, seed, form):
    from circuitgen import random_network
    from oracle import contract as C
    n = 6 + seed * 2
    net = random_network(n, 3 * n, 3, 100 + seed)
    m = seed % 4
    mu, pi, sched = oracle_schedule(net, m)
    want = C.brute_force_sum(n, net.tensors)
    _, vals = C.contract(net.tensors, sched)
    qm = qbe.Model(net.n_vars, net.tensors)
    _say(f"case random n={n} m={m} {form}")
    plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec=form)
    total, per = qbe.qbe_contract_slices(ctx, plan, 0, plan.n_slices, plan.workspace())
    assert rel(total, want) <= TOL
    check_slices(per, vals)


def test_wide_bucket_split_into_partial_products(qbe, ctx):
    """A variable shared by 11 tensors: its bucket has more operands than one
    per-step launch takes, so the plan multiplies them in two stages."""
    from oracle import contract as C
    rng = np.random.default_rng(7)
    tensors = []
    for i in range(1, 12):
        d = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
        tensors.append(((0, i), d))
    tensors.append(((3, 5, 7), rng.standard_normal((2, 2, 2)) + 0j))
    n = 12
    order = list(range(n))
    want = C.brute_force_sum(n, tensors)
    qm = qbe.Model(n, tensors)
    for form in ("per_step", "fused"):
        _say(f"case wide bucket {form}")
        plan = qbe.Plan(qm, order, [], ctx=ctx, exec=form)
        assert rel(qbe.qbe_contract(ctx, plan, plan.workspace()), want) <= TOL


def test_edge_cases(qbe, ctx):
    from oracle import contract as C
    rng = np.random.default_rng(3)
    # every variable sliced: no buckets at all, only scalar factors
    t = [((0, 1), rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))),
         ((1,), rng.standard_normal(2) + 0j)]
    want = C.brute_force_sum(2, t)
    qm = qbe.Model(2, t)
    for form in ("per_step", "fused"):
        _say(f"case all sliced {form}")
        plan = qbe.Plan(qm, [], [0, 1], ctx=ctx, exec=form)
        assert rel(qbe.qbe_contract(ctx, plan, plan.workspace()), want) <= TOL
    # a rank-0 tensor in the model and a single variable
    t2 = [((), np.array(2.0 - 1.0j)), ((0,), np.array([0.5, 1.5 + 1j]))]
    want2 = C.brute_force_sum(1, t2)
    qm2 = qbe.Model(1, t2)
    for form in ("per_step", "fused"):
        _say(f"case rank-0 input {form}")
        plan = qbe.Plan(qm2, [0], [], ctx=ctx, exec=form)
        assert rel(qbe.qbe_contract(ctx, plan, plan.workspace()), want2) <= TOL
    # a rank-12 tensor (a bucket above the per-step kernel's 8-bit tile)
    d = rng.standard_normal((2,) * 12) + 1j * rng.standard_normal((2,) * 12)
    t3 = [(tuple(range(12)), d), ((11, 12), rng.standard_normal((2, 2)) + 0j)]
    want3 = C.brute_force_sum(13, t3)
    qm3 = qbe.Model(13, t3)
    for form in ("per_step", "fused"):
        _say(f"case rank-12 {form}")
        plan = qbe.Plan(qm3, list(range(13)), [], ctx=ctx, exec=form)
        assert rel(qbe.qbe_contract(ctx, plan, plan.workspace()), want3) <= TOL


def test_ragged_slice_ranges_and_small_workspace(qbe, ctx):
    """Slice sub-ranges that do not divide the slice count, and a workspace
    that only holds a few slices (several slice groups per call)."""
    import torch
    from circuitgen import circuit_model, random_grid_circuit
    mod = circuit_model(random_grid_circuit(4, 5, 12, 3))
    mu, pi, sched = oracle_schedule(mod, 5)
    from oracle import contract as C
    _, vals = C.contract(mod.tensors, sched)
    qm = qbe.Model.from_circuitgen(mod)
    plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step")
    st = plan.stats()
    ws = torch.empty(st["ws_bytes_min"] + 3 * (st["ws_bytes_all_slices"] - st["ws_bytes_min"]) // 32,
                     dtype=torch.uint8, device="cuda")
    for (b, e) in [(0, 32), (3, 17), (31, 32), (5, 6)]:
        _say(f"case ragged range {b}-{e}")
        part, per = qbe.qbe_contract_slices(ctx, plan, b, e, ws)
        check_slices(per, vals[b:e])
        assert abs(part - sum(vals[b:e])) <= TOL * max(abs(sum(vals[b:e])), np.sqrt(np.mean(np.abs(vals) ** 2)))


def test_deterministic_bitwise(qbe, ctx):
    from circuitgen import circuit_model, random_grid_circuit
    mod = circuit_model(random_grid_circuit(5, 5, 16, 1))
    qm = qbe.Model.from_circuitgen(mod)
    _, mu, pi, _ = qbe.plan_circuit(qm, m=6)
    for form in ("fused", "per_step"):
        _say(f"case determinism {form}")
        plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec=form)
        ws = plan.workspace()
        a = qbe.qbe_contract_slices(ctx, plan, 0, 64, ws)
        b = qbe.qbe_contract_slices(ctx, plan, 0, 64, ws)
        assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_batch_of_uneven_instances(qbe, ctx):
    import torch
    from circuitgen import batch_instances, circuit_model, random_grid_circuit
    from oracle import contract as C
    inst = batch_instances(48)
    plans, wants = [], []
    for (r, c, d, m, seed) in inst:
        mod = circuit_model(random_grid_circuit(r, c, d, seed))
        mu, pi, sched = oracle_schedule(mod, m)
        wants.append(C.contract(mod.tensors, sched)[0])
        qm = qbe.Model.from_circuitgen(mod)
        plans.append(qbe.Plan(qm, pi, mu, ctx=ctx))
    _say("case batch of 48 instances (%d per-step)" % sum(p.stats()["exec"] == 1 for p in plans))
    batch = qbe.Batch(ctx, plans)
    ws = batch.workspace()
    amps = torch.zeros(2 * len(plans), dtype=torch.float64, device="cuda")
    batch.contract_async(ws, amps)
    torch.cuda.synchronize()
    got = amps.cpu().numpy().view(np.complex128)
    scale = [max(abs(w), 2.0 ** (-(r * c) / 2) * 1e-2) for w, (r, c, *_ ) in zip(wants, inst)]
    for g, w, s in zip(got, wants, scale):
        assert abs(g - w) <= TOL * s


def test_contract_batch_one_call(qbe, ctx):
    """qbe_contract_batch (transient batch, host amplitudes) against the
    oracle, its size query, and the too-small workspace error."""
    import torch
    from circuitgen import batch_instances, circuit_model, random_grid_circuit
    from oracle import contract as C
    inst = batch_instances(24)
    plans, wants = [], []
    for (r, c, d, m, seed) in inst:
        mod = circuit_model(random_grid_circuit(r, c, d, seed))
        mu, pi, sched = oracle_schedule(mod, m)
        wants.append(C.contract(mod.tensors, sched)[0])
        plans.append(qbe.Plan(qbe.Model.from_circuitgen(mod), pi, mu, ctx=ctx))
    _say("case one-call batch of 24 instances")
    need = qbe.qbe_contract_batch_workspace(ctx, plans)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    got = qbe.qbe_contract_batch(ctx, plans, ws)
    scale = [max(abs(w), 2.0 ** (-(r * c) / 2) * 1e-2) for w, (r, c, *_ ) in zip(wants, inst)]
    for g, w, s in zip(got, wants, scale):
        assert abs(g - w) <= TOL * s
    again = qbe.qbe_contract_batch(ctx, plans, ws)
    assert np.array_equal(got, again)
    with pytest.raises(qbe.QbeError, match="MEM_CAP"):
        qbe.qbe_contract_batch(ctx, plans, ws[: need - 16])


def test_unit_norm_over_all_bitstrings(qbe, ctx):
    """sum_x |<x|C|0>|^2 = 1 over all 2^9 bitstrings of a 3x3 circuit, one
    batch instance per bitstring."""
    import torch
    from circuitgen import circuit_model, random_grid_circuit
    circ = random_grid_circuit(3, 3, 8, 11)
    plans = []
    for x in range(1 << 9):
        qm = qbe.Model.from_circuitgen(circuit_model(circ, x))
        _, mu, pi, _ = qbe.plan_circuit(qm, m=1)
        plans.append(qbe.Plan(qm, pi, mu, ctx=ctx, exec="fused"))
    _say("case unit norm 3x3")
    batch = qbe.Batch(ctx, plans)
    amps = torch.zeros(2 * len(plans), dtype=torch.float64, device="cuda")
    batch.contract_async(batch.workspace(), amps)
    torch.cuda.synchronize()
    a = amps.cpu().numpy().view(np.complex128)
    assert abs(np.sum(np.abs(a) ** 2) - 1.0) <= 1e-5


def test_merged_launch_operand_holding_only_higher_summed_bits(qbe, ctx):
    """Batch instance 167 (5x6 depth 18, no slicing): its per-step plan has a
    merged launch with an operand that holds summed variables but not the
    first one and has more variables than the result."""
    from circuitgen import batch_instances, circuit_model, random_grid_circuit
    from oracle import contract as C
    r, c, d, m, seed = batch_instances(512)[167]
    mod = circuit_model(random_grid_circuit(r, c, d, seed))
    mu, pi, sched = oracle_schedule(mod, m)
    want = C.contract(mod.tensors, sched)[0]
    qm = qbe.Model.from_circuitgen(mod)
    _say(f"case batch instance 167 ({r}x{c} d{d} m{m}) per-step merged")
    for merge in (True, False):
        plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step", merge=merge)
        got = qbe.qbe_contract(ctx, plan, plan.workspace())
        assert abs(got - want) <= TOL * max(abs(want), 2.0 ** (-(r * c) / 2) * 1e-2)
