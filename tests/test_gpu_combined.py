"""The combined form: plans from the learned proposal (the elimination head
breaking greedy min-fill's ties, the slicing head as Alg. 2's score f)
contracted with split-BF16 products and fused or batched execution.  A plan
changes where the buckets are computed, never the sum (Eqs. 2-4): the
amplitudes must match the oracle's -- relative 1e-5 for FP32 and bf16x6, and
for bf16x3 the bound of its per-product residual (7 chained products of 4
split terms at 2.5 * 2^-17 each, as for the plain plans).  The network is
trained briefly here; any network gives a valid plan, so the bar is parity,
not plan quality (test_gpu_learned.py asserts the gains)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-5
BF16X3_BOUND = 7 * 4 * 2.5 * 2.0 ** -17


@pytest.fixture(scope="module")
def trained():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_10892_amd as qbe
    from paper_2004_10892_amd import learned as L
    from circuitgen import circuit_model, random_grid_circuit
    ctx = qbe.Context(0)
    circuits = [qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(5 + i % 2, 6, 14 + 2 * i, 7000 + i)))
                for i in range(10)]
    samples, n = L.make_dataset(circuits, seed=3, elim_states=2)
    print(f"case combined form: {n} labels", flush=True)
    net = qbe.Gnn(ctx, seed=7)
    L.train(net, samples, epochs=4, batch=8, lr=2e-3)
    return qbe, ctx, net


def learned_plan(qbe, net, qm, m):
    order, _, fell_back, _ = qbe.qbe_order_learned(qm, net, 16)
    mu, pi, tau = qbe.qbe_slice(qm, order, m, score="learned", net=net)
    return mu, pi, tau, fell_back


def test_learned_7x7_plan_with_fused_segments_in_three_precisions(trained):
    qbe, ctx, net = trained
    from circuitgen import circuit_model, random_grid_circuit
    g = json.load(open(os.path.join(GOLD, "amplitudes.json")))["grid7x7_d24_m10"]
    qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(7, 7, 24, g["seed"])))
    want = complex(*g["oracle"])
    mu, pi, tau, fell_back = learned_plan(qbe, net, qm, 10)
    assert len(mu) == 10
    print(f"case combined 7x7 d24: width {tau}, order from "
          f"{'min-fill (fallback)' if fell_back else 'the elimination head'}", flush=True)
    for prec in ("fp32", "bf16x6", "bf16x3"):
        plan = qbe.Plan(qm, pi, mu, ctx=ctx, exec="per_step", precision=prec, fused_prefix=True,
                        fused_segments=True)
        got = qbe.qbe_contract(ctx, plan, plan.workspace())
        err = abs(got - want) / abs(want)
        print(f"  {prec}: rel err {err:.2e}, {plan.stats()['n_launches']} launches", flush=True)
        assert err <= (BF16X3_BOUND if prec == "bf16x3" else TOL), (prec, err)


@pytest.mark.parametrize("exec_form,prec", [("auto", "fp32"), ("per_step", "bf16x6"), ("per_step", "bf16x3")])
def test_learned_plans_of_batch_instances_in_one_batch(trained, exec_form, prec):
    """The first 48 instances of the 512-instance workload, each planned by
    the learned proposal at its own m, in one batched call, against the
    oracle's stored amplitudes on the scale max(|a|, 0.1 * 2^(-n/2)) (the
    near-zero reading of the batch test)."""
    import torch
    qbe, ctx, net = trained
    from circuitgen import circuit_model, random_grid_circuit
    gold = json.load(open(os.path.join(GOLD, "batch512.json")))["instances"][:48]
    plans = []
    for x in gold:
        qm = qbe.Model.from_circuitgen(circuit_model(random_grid_circuit(x["rows"], x["cols"], x["depth"], x["seed"])))
        mu, pi, _, _ = learned_plan(qbe, net, qm, x["m"])
        plans.append(qbe.Plan(qm, pi, mu, ctx=ctx, exec=exec_form, precision=prec))
    print(f"case combined batch of 48 learned plans, {exec_form} {prec}", flush=True)
    batch = qbe.Batch(ctx, plans)
    amps = torch.zeros(2 * len(plans), dtype=torch.float64, device="cuda")
    batch.contract_async(batch.workspace(), amps)
    torch.cuda.synchronize()
    got = amps.cpu().numpy().view(np.complex128)
    want = np.array([complex(*x["oracle"]) for x in gold])
    scale = np.array([max(abs(complex(*x["oracle"])), 0.1 * 2.0 ** (-(x["rows"] * x["cols"]) / 2)) for x in gold])
    err = np.abs(got - want) / scale
    print(f"  max scaled error {err.max():.2e}", flush=True)
    assert np.all(err <= (BF16X3_BOUND if prec == "bf16x3" else TOL)), (int(err.argmax()), float(err.max()))
